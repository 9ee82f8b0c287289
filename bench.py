"""Throughput of the GGEM slit evaluation on one MI355X.

Workload (default): single layer on 50 capsule meshes (unit spheres, 642 nodes
each, 32,100 nodal point forces, force-free per capsule) in a 20 x 10 x 20
slit (walls at y = +-5), alpha = 2, r_c = 2, grid 128 x 128 Fourier x 65
Chebyshev; targets = sources.  A step is one full evaluation (binning, local
sum, wall data, spread, forward FFT + Chebyshev, tau solves, inverse
transforms, interpolation) on inputs resident in device memory.

Prints one JSON line: throughput in Mpoints/s (points = targets) for the
mixed-precision path, with its error against the FP64 path on the same GPU,
the FP64 path's throughput, the dominant kernel's roofline, the Fredholm
solve time to a relative residual of 1e-6 on 100 drops in shear (plain and
learned warm starts) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6

# Algorithmic work per unit (flops), counted per pair within r_c (local sum)
# and per (source, grid node within r_c) update (spread).
FLOP_NEAR_SL = 50.0
FLOP_NEAR_DL = 65.0
FLOP_SPREAD = 12.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--workload", choices=["capsules_sl", "capsules_dl", "batched"],
                    default="capsules_sl")
    ap.add_argument("--branches", type=int, default=0,
                    help="streams of the batched workload (0: autotuned, cached on disk)")
    ap.add_argument("--roofline-stage", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serialized", action="store_true",
                    help="time one evaluation captured into a HIP graph on a single stream "
                         "(no second stream: every kernel runs alone) and replayed; for "
                         "per-kernel profiles, not the headline figure")
    ap.add_argument("--cpu-capsules", type=int, default=5)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device three times (a "
                         "plain copy of known size, to scale HBM counters)")
    ap.add_argument("--fredholm-steps", type=int, default=200,
                    help="time steps of the drop run behind the Fredholm figures (0: skip)")
    return ap.parse_args()


def time_steps(plan, call, steps, warmup, stage=None):
    import torch
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    if stage is not None:
        plan.time_stage(stage, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.status()
    stage_ms = None
    if stage is not None:
        tot, n = plan.stage_time()
        stage_ms = tot / max(n, 1)
        plan.time_stage(-1, 1)
    return (t1 - t0) * 1e3 / steps, stage_ms


def measured_traffic(stage, workload, precision):
    """HBM bytes per launch of the stage's kernel from the committed counter
    runs (profiles/traffic.json), or None when there are none for this
    workload or the kernel's source has changed since they were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            ent = json.load(fh).get(stage)
    except (OSError, ValueError):
        return None
    if not ent or ent.get("workload") != workload or ent.get("precision") != precision:
        return None
    with open(os.path.join(ROOT, ent["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != ent["sha256"]:
            return None
    return int(ent["bytes_per_launch"])


def cpu_baseline(c, ncap):
    """FP64 oracle on the first `ncap` capsules (same box and grid)."""
    import oracle as O
    nv = c.meta.get("nv") or c.meta.get("ng")
    n = ncap * nv
    g = O.SlitGrid.from_case(c)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    if c.normals is None:
        O.single_layer(g, c.xs[:n], c.f[:n], c.xt[:n])
    else:
        O.double_layer(g, c.xs[:n], c.f[:n], c.xt[:n], c.normals[:n])
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return {
        "value": n / wall / 1e6,
        "unit": "Mpoints/s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": f"{ncap} of {c.meta['ncap']} capsules ({n} points as sources and targets) on "
                  f"the full {c.Nx}x{c.Nz}x{c.Ny} grid, FP64 NumPy oracle, wall {wall:.1f} s, "
                  f"cpu {cpu:.1f} s",
    }


def fredholm(steps):
    """Seconds per Fredholm solve to 1e-6 on 100 drops in shear (64,200 nodes,
    192,600 unknowns, 384,000 Gauss-point sources): the drop run, training of
    the warm-start network on its first 3/4 and every start on the rest."""
    from paper_1109_6587_amd.warmstart import run
    from workloads import case_shear_drops
    train = (3 * steps) // 4
    res, _ = run(case_shear_drops(4), steps=steps, train_steps=train,
                 log=lambda m: print(m, file=sys.stderr, flush=True))
    st = res["starts"]
    return {
        "metric": "Fredholm solve s to 1e-6",
        "value": round(st["learned_judged"]["seconds_mean"], 5),
        "plain_warm_start_s": round(st["plain"]["seconds_mean"], 5),
        "unit": "s",
        "products": {k: v["products_mean"] for k, v in st.items()},
        "seconds": {k: round(v["seconds_mean"], 5) for k, v in st.items()},
        "speedup_learned_vs_plain": round(res["speedup_vs_plain"], 4),
        "products_saved_per_solve": round(res["products_saved_per_solve"], 3),
        "prediction_rel_err": round(res["prediction_rel_err_mean"], 4),
        "workload": res["workload"], "unknowns": res["unknowns"], "sources": res["sources"],
        "precision": res["precision"], "train_solves": res["train_solves"],
        "test_solves": res["test_solves"], "simulation_s": res["simulation_s"],
        "training_s": res["training_s"],
    }


def bench_batched(args):
    """48 independent instances (1.5M points) as one captured graph per step."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    from workloads import case_batched

    dev = torch.device("cuda:0")
    cases = case_batched(3)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    so = np.concatenate([[0], np.cumsum([c.ns for c in cases])])
    to = np.concatenate([[0], np.cumsum([c.nt for c in cases])])
    xs = t(np.concatenate([c.xs for c in cases]))
    f = t(np.concatenate([c.f for c in cases]))
    n = int(to[-1])
    out = {p: torch.empty((n, 3), dtype=torch.float64, device=dev) for p in ("mixed", "fp64")}
    branches, tuned_ms, cached = args.branches, None, None
    if branches <= 0:
        from paper_1109_6587_amd.autotune import tune_batch
        branches, tuned_ms, cached = tune_batch(
            cases, (so, xs, f, to, xs, out[args.precision]), precision=args.precision,
            log=lambda m: print(m, file=sys.stderr, flush=True))
    batches = {p: G.Batch(cases, precision=p, n_branches=branches) for p in out}
    for p, b in batches.items():
        b.capture(so, xs, f, to, xs, out[p])
        b.replay()
        b.status()
    err = float(torch.linalg.norm(out["mixed"] - out["fp64"]) / torch.linalg.norm(out["fp64"]))

    def timed(b, steps):
        for _ in range(args.warmup):
            b.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    prec = args.precision
    other = "fp64" if prec == "mixed" else "mixed"
    ms = timed(batches[prec], args.steps)
    ms_other = timed(batches[other], max(10, args.steps // 4))
    batches[prec].status()
    # eager submission of the same batch, for the graph's launch saving
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        batches[prec].single_layer(so, xs, f, to, xs, out[prec])
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / 10
    line = {
        "metric": "GGEM Mpoints/s (mixed vs FP64, rel err 1e-5); Fredholm solve s to 1e-6",
        "value": round(n / (ms * 1e-3) / 1e6, 3), "unit": "Mpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "batched_48", "instances": len(cases), "points": n,
                   "precision": prec, "branches": branches, "submission": "hip graph"},
        "autotune": {"ms_by_branches": tuned_ms, "from_cache": cached},
        "err_vs_fp64": {"rel_l2": err},
        f"{other}_ms_per_step": round(ms_other, 5),
        "eager_ms_per_step": round(ms_eager, 5),
        "roofline": None,
    }
    print(json.dumps(line))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
    else:
        bench_single(args)
    if args.calibrate_copy > 0:
        import torch
        n = args.calibrate_copy * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration: copied {n} bytes three times", file=sys.stderr)


def bench_single(args):
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    from workloads import case_capsules_dl, case_capsules_sl

    dev = torch.device("cuda:0")
    c = case_capsules_sl(1) if args.workload == "capsules_sl" else case_capsules_dl(2)
    dl = c.normals is not None
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xs, f = t(c.xs), t(c.f)
    # the capsule workloads evaluate at their own sources: passing the same
    # array lets the library reuse the source binning for the targets
    xt = xs if np.array_equal(c.xt, c.xs) else t(c.xt)
    nrm = t(c.normals) if dl else None
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=dev)

    plans = {p: G.Plan.from_case(c, precision=p, sync_checks=False) for p in ("mixed", "fp64")}

    def caller(plan):
        if dl:
            return lambda: plan.double_layer(xs, f, xt, nrm, out=out)
        return lambda: plan.single_layer(xs, f, xt, out=out)

    # accuracy of the mixed path against the FP64 path (same inputs)
    caller(plans["fp64"])()
    ref = out.clone()
    caller(plans["mixed"])()
    torch.cuda.synchronize()
    err_l2 = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
    err_max = float((out - ref).abs().max() / ref.abs().max())

    plan = plans[args.precision]
    if args.serialized:
        return bench_serialized(args, c, plan, caller(plan), err_l2, err_max)
    caller(plan)()
    near_pairs, spread_pairs = plan.work()
    stage = args.roofline_stage
    if stage == "auto":
        # the dominant of the two pair kernels, timed before the measured region
        per = {}
        for st in ("near", "spread"):
            _, per[st] = time_steps(plan, caller(plan), 10, 2, stage=st)
        stage = max(per, key=per.get)
    ms, stage_ms = time_steps(plan, caller(plan), args.steps, args.warmup, stage=stage)
    other = "fp64" if args.precision == "mixed" else "mixed"
    ms_other, _ = time_steps(plans[other], caller(plans[other]), max(10, args.steps // 4),
                             args.warmup)
    value = c.nt / (ms * 1e-3) / 1e6

    if stage == "near":
        flops = near_pairs * (FLOP_NEAR_DL if dl else FLOP_NEAR_SL)
    elif stage == "spread":
        flops = spread_pairs * FLOP_SPREAD
    else:
        flops = None
    peak = PEAK_FP32_TFLOPS if args.precision == "mixed" else PEAK_FP64_TFLOPS
    roof = None
    if flops is not None and stage_ms:
        ach = flops / (stage_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4),
                "traffic": measured_traffic(stage, c.name, args.precision), "kernel": stage,
                "kernel_ms": round(stage_ms, 5), "work_units": near_pairs if stage == "near" else spread_pairs}

    line = {
        "metric": "GGEM Mpoints/s (mixed vs FP64, rel err 1e-5); Fredholm solve s to 1e-6",
        "value": round(value, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": c.name, "points": c.nt, "sources": c.ns,
                   "grid": [c.Nx, c.Nz, c.Ny], "alpha": c.alpha, "rc": c.rc,
                   "box": [c.Lx, 2 * c.H, c.Lz], "precision": args.precision,
                   "layer": "double" if dl else "single"},
        "err_vs_fp64": {"rel_l2": err_l2, "rel_max": err_max},
        f"{other}_mpoints_per_s": round(c.nt / (ms_other * 1e-3) / 1e6, 3),
        f"{other}_ms_per_step": round(ms_other, 5),
        "work": {"near_pairs": near_pairs, "spread_updates": spread_pairs},
        "roofline": roof,
    }
    if args.fredholm_steps > 0:
        line["fredholm"] = fredholm(args.fredholm_steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c, args.cpu_capsules)
    print(json.dumps(line))


def bench_serialized(args, c, plan, call, err_l2, err_max):
    import torch
    s = torch.cuda.Stream()
    plan.set_stream(s)
    with torch.cuda.stream(s):
        call()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        call()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    plan.status()
    print(json.dumps({
        "metric": "GGEM Mpoints/s, one evaluation per graph replay on a single stream",
        "value": round(c.nt / (ms * 1e-3) / 1e6, 3), "unit": "Mpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": c.name, "points": c.nt, "grid": [c.Nx, c.Nz, c.Ny],
                   "precision": args.precision, "mode": "serialized graph"},
        "err_vs_fp64": {"rel_l2": err_l2, "rel_max": err_max}}))


if __name__ == "__main__":
    main()
