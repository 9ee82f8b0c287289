"""Learned warm start for the Fredholm solves of a drop suspension in shear.

1. Run the suspension (``drops.DropSuspension``) and keep, for every solve,
   the shape (positions, normals, Lap x), the right-hand side, the previous
   stage's density (the plain warm start) and the converged density.
2. Train the per-node network (ggem_mlp_*) on the solves of the first
   `train_steps` steps to predict what linear extrapolation of the density
   misses, q - (q_prev + dq_prev) (dq_prev: the last change of the density),
   from the node features (position relative to the drop centroid, normal,
   curvature term, previous density and its last change).
3. On every solve of the remaining steps, solve from the same recorded
   state with each start and report products and times:
   plain (previous density, the paper's start), extrapolated (previous
   density plus its last change), learned_direct (the extrapolation plus the
   prediction), learned_blend (ggem_fredholm_solve_guided from the
   extrapolation on every solve: the least-squares step along the
   prediction, never worse than the extrapolation, one extra product) and
   learned_judged (the deployed rule: every `judge_every`-th solve is a
   guided one whose step c judges the network against the extrapolated
   start; the solves in between start from the extrapolation plus the
   prediction while the last c >= 1/2, else from the extrapolation).

Data preparation (the two normalisation scalars and the target differences)
uses torch tensor operations; the network's features, forward and backward
passes, Adam updates and predictions run in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import ggem as B
from .drops import DropSuspension


class Recorder:
    """Keeps every solve of a run on the device."""

    def __init__(self):
        self.solves = []
        self._cur = None

    def before(self, x, nrm, lap, b, q0, stage):
        self._cur = dict(x=x.clone(), nrm=nrm.clone(), lap=lap.clone(), b=b.clone(),
                         q_prev=q0.clone(), stage=stage)

    def after(self, q):
        self._cur["q"] = q.clone()
        self.solves.append(self._cur)
        self._cur = None


def he_uniform(seed):
    """Initial parameters, packed as ggem_mlp_set_params expects (He-uniform
    weights drawn layer by layer with numpy's default_rng(seed), zero biases)."""
    rng = np.random.default_rng(seed)
    sizes = (B.MLP_IN, B.MLP_HIDDEN, B.MLP_HIDDEN, B.MLP_HIDDEN, B.MLP_OUT)
    parts = []
    for i in range(4):
        a = np.sqrt(6.0 / sizes[i])
        parts.append(rng.uniform(-a, a, size=(sizes[i + 1], sizes[i])).ravel())
        parts.append(np.zeros(sizes[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def run(case, steps=200, train_steps=150, precision="mixed", tol=1e-6, restart=20, epochs=3,
        batch=8192, lr=1e-3, seed=0, judge_every=4, log=print):
    import torch

    dev = torch.device("cuda:0")
    sim = DropSuspension(case, precision=precision, restart=restart, tol=tol)
    rec = Recorder()
    t0 = time.perf_counter()
    for s in range(steps):
        sim.step(hook=rec)
        if s % 25 == 0 or s == steps - 1:
            r = sim.records[-1]
            log(f"step {s}: products {r.iters}, rel_res {r.rel_res:.2e}, {r.seconds * 1e3:.1f} ms")
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    n = case.nodes.shape[0]
    S = rec.solves
    # last change of the density before each solve (zero before the second)
    for k, sv in enumerate(S):
        sv["dq_prev"] = (S[k - 1]["q"] - S[k - 1]["q_prev"]) if k >= 2 else torch.zeros_like(sv["q"])
    first = 2                       # the first two solves start cold
    ntrain = 2 * train_steps
    train, test = S[first:ntrain], S[ntrain:]

    # normalisation from the training solves; the target is the residual of
    # linear extrapolation
    resid = lambda sv: sv["q"] - sv["q_prev"] - sv["dq_prev"]  # noqa: E731
    with torch.no_grad():
        c_all = torch.cat([-(sv["lap"] * sv["nrm"]).sum(1) for sv in train])
        qp_all = torch.cat([sv["q_prev"] for sv in train])
        dq_all = torch.cat([sv["q"] - sv["q_prev"] for sv in train])
        r_all = torch.cat([resid(sv) for sv in train])
        s_c = 1.0 / float(c_all.pow(2).mean().sqrt())
        s_q = 1.0 / float(qp_all.pow(2).mean().sqrt())
        sigma = float(dq_all.pow(2).mean().sqrt())
        sigma_r = float(r_all.pow(2).mean().sqrt())
        del c_all, qp_all, dq_all, r_all
    scales = [1.0] * 6 + [s_c] + [s_q] * 3 + [1.0 / sigma] * 3
    mlp = B.MLP(max(n, batch), torch.as_tensor(he_uniform(seed), device=dev))
    X = {k: mlp.features(sv["x"], sv["nrm"], sv["lap"], sv["q_prev"], sv["dq_prev"], case.nv,
                         scales)
         for k, sv in enumerate(S) if k >= first}
    T = {k: (resid(S[k]) / sigma_r).float().contiguous() for k in range(first, ntrain)}

    # training: mini-batches of `batch` consecutive nodes of one solve, in a
    # seeded random order; learning rate decays linearly to lr/10
    rng = np.random.default_rng(seed + 1)
    chunks = [(k, a) for k in range(first, ntrain) for a in range(0, n, batch)]
    t1 = time.perf_counter()
    nstep = epochs * len(chunks)
    it = 0
    for ep in range(epochs):
        for j in rng.permutation(len(chunks)):
            k, a = chunks[j]
            e = min(n, a + batch)
            mlp.train_step(X[k][a:e], T[k][a:e], lr * (1.0 - 0.9 * it / nstep))
            it += 1
        loss = float(np.mean([mlp.gradients(X[k], T[k])[0] for k in range(first, ntrain, 15)]))
        log(f"epoch {ep}: training loss {loss:.4f} (fraction of the target variance)")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1

    # evaluation on the held-out solves, every start from the same recorded state
    names = ("plain", "extrapolated", "learned_direct", "learned_blend", "learned_judged")
    res_it = {m: [] for m in names}
    res_t = {m: [] for m in names}
    pred_err, extrap_err, blend = [], [], []
    use_learned = True
    for k in range(ntrain, len(S)):
        sv = S[k]
        surf = B.Surface(sv["x"], sv["nrm"], sim.tri, sim.kappa)
        true = sv["q"] - sv["q_prev"]
        for m in names:
            torch.cuda.synchronize()
            ta = time.perf_counter()
            q = sv["q_prev"].clone()
            extra = 0
            if m == "plain":
                its, rr = sim.solver.solve(surf, sv["b"], q, tol=tol, max_iter=sim.max_iter)
            else:
                # linear extrapolation, the base of every other start
                sim.solver.advance(sv["q_prev"], sv["dq_prev"], 1.0, out=q)
                if m == "extrapolated":
                    its, rr = sim.solver.solve(surf, sv["b"], q, tol=tol, max_iter=sim.max_iter)
                else:
                    dq = mlp.predict(X[k], sigma_r)
                    judged_now = m == "learned_judged" and (k - ntrain) % judge_every == 0
                    if m == "learned_blend" or judged_now:
                        its, rr, c = sim.solver.solve_guided(surf, sv["b"], q, dq, tol=tol,
                                                             max_iter=sim.max_iter)
                        extra = 1
                        if judged_now:
                            use_learned = c >= 0.5
                        else:
                            blend.append(c)
                    elif m == "learned_direct" or use_learned:
                        sim.solver.advance(q, dq, 1.0, out=q)
                        its, rr = sim.solver.solve(surf, sv["b"], q, tol=tol,
                                                   max_iter=sim.max_iter)
                    else:
                        its, rr = sim.solver.solve(surf, sv["b"], q, tol=tol,
                                                   max_iter=sim.max_iter)
                    if m == "learned_direct":
                        nt = float(torch.linalg.norm(true))
                        pred_err.append(float(torch.linalg.norm(sv["dq_prev"] + dq - true)) / nt)
                        extrap_err.append(float(torch.linalg.norm(sv["dq_prev"] - true)) / nt)
            torch.cuda.synchronize()
            res_t[m].append(time.perf_counter() - ta)
            res_it[m].append(its + extra)
            if rr > tol:
                raise RuntimeError(f"evaluation solve {k} ({m}) stalled at {rr:.2e}")
    summary = {m: {"products_mean": float(np.mean(res_it[m])),
                   "seconds_mean": float(np.mean(res_t[m]))} for m in names}
    res = {
        "workload": case.name, "nodes": n, "unknowns": 3 * n, "sources": 3 * case.tri.shape[0],
        "precision": precision, "tol": tol, "solves_total": len(S),
        "train_solves": len(train), "test_solves": len(test),
        "simulation_s": round(t_sim, 3), "training_s": round(t_train, 3),
        "train_minibatches": nstep, "judge_every": judge_every,
        "starts": summary,
        "prediction_rel_err_mean": float(np.mean(pred_err)),
        "extrapolation_rel_err_mean": float(np.mean(extrap_err)),
        "blend_step_mean": float(np.mean(blend)),
        "products_saved_per_solve": summary["plain"]["products_mean"]
        - summary["learned_judged"]["products_mean"],
        "products_saved_vs_extrapolated": summary["extrapolated"]["products_mean"]
        - summary["learned_judged"]["products_mean"],
        "speedup_vs_plain": summary["plain"]["seconds_mean"] / summary["learned_judged"]["seconds_mean"],
        "speedup_vs_extrapolated": summary["extrapolated"]["seconds_mean"]
        / summary["learned_judged"]["seconds_mean"],
    }
    return res, sim


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--train-steps", type=int, default=150)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--precision", default="mixed")
    args = ap.parse_args()
    from workloads import case_shear_drops
    res, _ = run(case_shear_drops(4), steps=args.steps, train_steps=args.train_steps,
                 epochs=args.epochs, precision=args.precision,
                 log=lambda m: print(m, flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
