"""Throughput of the GGEM slit evaluation on one MI355X.

Headline workload: the double layer (stresslet, traction n . sigma at the
targets) on 400 capsule meshes -- unit spheres of 1,280 triangles with three
interior Gauss points each, 1,536,000 point force-dipole strengths q times
the Gauss weight, targets = sources with the triangles' outward normals --
in a 40 x 12 x 40 slit (walls at y = +-6), alpha = 2, r_c = 2, grid
256 x 256 Fourier x 65 Chebyshev.  A step is one full evaluation (binning,
local sum, wall data and pressure gauge, spread, forward FFT + Chebyshev,
tau solves, stress assembly, inverse transforms, interpolation) on inputs
resident in device memory; the value is targets per second in mixed
precision.

The JSON line also carries: the FP64 path's throughput on the same GPU and
the mixed path's error against it; the error of each path against FP64
oracle values stored for 256 sampled targets (total, local and global
parts); the dominant kernel's roofline (the local sum) with the spread's
beside it; the CPU oracle timed on a bounded sample; and extra workloads --
64 forces + 1,000 probes (microseconds per call), the 50-capsule single
layer, the 48-instance batch replayed as one HIP graph, the Fredholm solve
time to a relative residual of 1e-6 on 100 drops in shear with and without
the learned warm start, the rigid-sphere validation, the spectral off-mesh
evaluation beside the Lagrange stencil, the stage time of neo-Hookean
capsule suspensions (15 to 120 capsules, three viscosity ratios), and
velocity, pressure and stress at probes.
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import statistics
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

METRIC = "GGEM Mpoints/s (mixed vs FP64, rel err 1e-5); Fredholm solve s to 1e-6"
EXTRAS = ("small", "capsules_sl", "batched", "fredholm", "rigid", "spectral", "capsules",
          "probes", "convergence")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["mixed", "fp64", "mixed_bf16"], default="mixed")
    ap.add_argument("--workload", choices=["capsules_dl", "capsules_sl", "batched", "extras"],
                    default="capsules_dl",
                    help="'extras': only the extra workloads of --extras, as one JSON line "
                         "(for per-workload profiles), without the headline evaluation")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated extra workloads in the line: "
                         f"{', '.join(EXTRAS)}, or 'none'")
    ap.add_argument("--branches", type=int, default=0,
                    help="streams of the batched workload (0: autotuned, cached on disk)")
    ap.add_argument("--roofline-stage", default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 comparison path (profiling runs)")
    ap.add_argument("--serialized", action="store_true",
                    help="time one evaluation captured into a HIP graph on a single stream "
                         "(no second stream: every kernel runs alone) and replayed; for "
                         "per-kernel profiles, not the headline figure")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device three times (a "
                         "plain copy of known size, to scale HBM counters)")
    ap.add_argument("--fredholm-steps", type=int, default=200,
                    help="time steps of the drop run behind the Fredholm figures")
    return ap.parse_args()


def time_steps(plan, call, steps, warmup, stage=None):
    """Mean ms per call over `steps` calls after `warmup`, and the mean
    duration of `stage` from HIP events the library records around that
    stage's launches on the stream it runs on."""
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
            ent = json.load(fh).get(f"{workload}:{stage}")
    except (OSError, ValueError):
        return None
    if not ent or ent.get("precision") != precision:
        return None
    with open(os.path.join(ROOT, ent["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != ent["sha256"]:
            return None
    return int(ent["bytes_per_launch"])


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    import numpy as np
    return float(np.abs(a - b).max() / np.abs(b).max())


def golden(c):
    """FP64 oracle values at 256 sampled targets (tests/golden), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{c.name}_sampled.json")
    try:
        with open(path) as fh:
            ref = json.load(fh)
    except OSError:
        return None
    if ref.get("seed") != c.meta.get("seed") or ref.get("grid") != [c.Nx, c.Nz, c.Ny]:
        return None
    return ref


def cpu_baseline(c, budget_targets=16, spread_sources=1000, interp_frac=0.01):
    """The FP64 NumPy oracle timed stage by stage on a bounded sample of the
    workload and extrapolated linearly to the whole of it: the local sum on
    `budget_targets` seeded targets (brute force over all sources), the wall
    data on as many wall nodes, the spread on `spread_sources` seeded
    sources; the grid stages (forward transforms, per-mode solves, stress or
    velocity assembly, inverse transforms) in full; the interpolation on a
    seeded `interp_frac` of the targets."""
    import numpy as np

    import oracle as O
    from oracle import ggem as OG
    g = O.SlitGrid.from_case(c)
    dl = c.normals is not None
    rng = np.random.default_rng(17)
    xs, xt = g.wrap(c.xs), g.wrap(c.xt)
    q = np.asarray(c.f, dtype=np.float64)
    times = {}
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    w0 = time.perf_counter()

    def clock(name, fn, scale):
        t0 = time.perf_counter()
        out = fn()
        times[name] = (time.perf_counter() - t0) * scale
        return out

    sel = np.sort(rng.choice(c.nt, size=min(budget_targets, c.nt), replace=False))
    if dl:
        clock("local", lambda: OG.local_traction(g, xs, q, xt[sel], c.normals[sel]),
              c.nt / sel.size)
    else:
        clock("local", lambda: OG.local_velocity(g, xs, q, xt[sel]), c.nt / sel.size)
    nwall = 2 * g.Nx * g.Nz
    wsel = rng.choice(nwall, size=min(budget_targets, nwall), replace=False)
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    wpts = np.concatenate([np.stack([X.ravel(), np.full(X.size, yw), Z.ravel()], axis=1)
                           for yw in (-g.H, g.H)])
    clock("wall", lambda: OG.local_velocity(g, xs, q, wpts[wsel]), nwall / wsel.size)
    if dl:
        clock("gauge", lambda: OG.pressure_gauge(g, xs, q), 1.0)
    ssel = np.sort(rng.choice(c.ns, size=min(spread_sources, c.ns), replace=False))
    F = clock("spread", lambda: OG.spread(g, xs[ssel], q[ssel]), c.ns / ssel.size)
    Cf, Ci = OG.cheb_forward_matrix(g.Ny), OG.cheb_inverse_matrix(g.Ny)
    D = OG.cheb_diff_matrix(g.Ny)
    zw = np.zeros((3, g.Nx, g.Nz))

    def forward():
        return (OG._apply_y(Cf, OG.dft_xz(g, F)), OG.dft_xz(g, zw), OG.dft_xz(g, zw))

    Fh, gm, gp = clock("fft_cheb_fwd", forward, 1.0)
    u, v, w, p = clock("tau", lambda: OG.solve_modes(g, Fh, gm, gp, 0.0), 1.0)

    def inverse():
        if not dl:
            return np.stack([OG.idft_xz(g, OG._apply_y(Ci, a)) for a in (u, v, w)])
        ikx = 1j * g.kx[None, :, None]
        ikz = 1j * g.kz[None, None, :]
        dy = lambda a: OG._apply_y(D, a) / g.H  # noqa: E731
        sig = (-p + 2.0 * ikx * u, -p + 2.0 * dy(v), -p + 2.0 * ikz * w,
               dy(u) + ikx * v, ikz * u + ikx * w, ikz * v + dy(w))
        return np.stack([OG.idft_xz(g, OG._apply_y(Ci, a)) for a in sig])

    fields = clock("cheb_fft_inv", inverse, 1.0)
    isel = np.sort(rng.choice(c.nt, size=max(1, int(interp_frac * c.nt)), replace=False))
    clock("interp", lambda: OG.interpolate(g, fields, xt[isel]), c.nt / isel.size)
    wall_s = time.perf_counter() - w0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu_s = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    total = sum(times.values())
    return {
        "value": c.nt / total / 1e6,
        "unit": "Mpoints/s",
        "cores": max(1, int(round(cpu_s / wall_s))),
        "kind": "oracle",
        "extrapolated": True,
        "seconds_per_evaluation": round(total, 2),
        "stage_seconds": {k: round(v, 3) for k, v in times.items()},
        "sample": (f"FP64 NumPy oracle, stage by stage, extrapolated linearly to the whole "
                   f"workload ({c.nt} targets, {c.ns} sources): local sum on {sel.size} seeded "
                   f"targets and wall data on {wsel.size} of {nwall} wall nodes (brute force "
                   f"over all sources), spread on {ssel.size} seeded sources, grid stages on the "
                   f"full {c.Nx}x{c.Nz}x{c.Ny} grid, interpolation on {isel.size} targets; "
                   f"wall {wall_s:.1f} s, cpu {cpu_s:.1f} s"),
    }


def roofline_entry(stage, stage_ms, work_units, flop, peak, traffic):
    ach = work_units * flop / (stage_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "traffic": traffic, "kernel": stage,
            "kernel_ms": round(stage_ms, 5), "work_units": int(work_units),
            "flop_per_unit": flop}


def step_roofline(c, precision, dl, near_units, spread_units, ms):
    """Whole-step roofline: T_ideal = sum over the stages of max(flop /
    peak, bytes / 8 TB/s) with the kernel-counted pairs and updates (the local
    sum and the spread are ALU-bound) and the grid stages' algorithmic bytes
    (each field read and written once per pass: z and x FFTs, Chebyshev
    products, tau coefficients in and out, interpolation); the fraction is
    T_ideal / T_measured.  The wall data's local sum and the binning are left
    out (a smaller T_ideal, a lower fraction)."""
    fp64 = precision == "fp64"
    peak = (PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS) * 1e12
    e = 8 if fp64 else 4
    nf = 6 if dl else 3
    n3 = c.Ny * c.Nx * c.Nz                  # real nodes per field
    nh = c.Ny * c.Nx * (c.Nz // 2 + 1)       # complex coefficients per field
    grid = {
        "fft_fwd": 3 * (n3 * e + nh * 2 * e) + 3 * (2 * nh * 2 * e),
        "cheb_fwd": 3 * 2 * nh * 2 * e,
        "tau": 3 * nh * 2 * e + nf * nh * 2 * e,
        "cheb_inv": nf * 2 * nh * 2 * e,
        "fft_inv": nf * (2 * nh * 2 * e) + nf * (nh * 2 * e + n3 * e),
        "interp": nf * n3 * e + c.nt * 24,
    }
    terms = {"near": near_units * (FLOP_NEAR_DL if dl else FLOP_NEAR_SL) / peak * 1e3,
             "spread": spread_units * FLOP_SPREAD / peak * 1e3}
    terms.update({k: v / (PEAK_HBM_GBS * 1e9) * 1e3 for k, v in grid.items()})
    t = sum(terms.values())
    return {"t_ideal_ms": round(t, 4), "t_measured_ms": round(ms, 4), "frac": round(t / ms, 4),
            "terms_ms": {k: round(v, 4) for k, v in terms.items()},
            "grid_bytes": sum(grid.values())}


def measure_case(c, args, precision, with_other=True, golden_parts=True):
    """Mixed (or FP64) evaluation of one case: throughput, the roofline of
    the local sum and of the spread, errors against the other precision and
    against the stored oracle sample."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G

    dev = torch.device("cuda:0")
    dl = c.normals is not None
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xs, f = t(c.xs), t(c.f)
    # the capsule workloads evaluate at their own sources: passing the same
    # array lets the library reuse the source binning for the targets
    xt = xs if np.array_equal(c.xt, c.xs) else t(c.xt)
    nrm = t(c.normals) if dl else None
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=dev)
    other = "fp64" if precision == "mixed" else "mixed"
    precs = (precision, other) if with_other else (precision,)
    plans = {p: G.Plan.from_case(c, precision=p, sync_checks=False) for p in precs}

    def caller(plan, parts=G.PART_ALL):
        if dl:
            return lambda: plan.double_layer(xs, f, xt, nrm, parts=parts, out=out)
        return lambda: plan.single_layer(xs, f, xt, parts=parts, out=out)

    res = {}
    ref = golden(c)
    outs = {}
    for p in precs:
        caller(plans[p])()
        plans[p].status()
        outs[p] = out.cpu().numpy()
    if ref is not None:
        sel = np.asarray(ref["targets"])
        err = {}
        for p in precs:
            e = {"total": {"rel_l2": rel_l2(outs[p][sel], np.asarray(ref["total"])),
                           "rel_max": rel_max(outs[p][sel], np.asarray(ref["total"]))}}
            if golden_parts:
                for key, parts in (("local", G.PART_LOCAL), ("global", G.PART_GLOBAL)):
                    caller(plans[p], parts)()
                    plans[p].status()
                    o = out.cpu().numpy()[sel]
                    e[key] = {"rel_l2": rel_l2(o, np.asarray(ref[key])),
                              "rel_max": rel_max(o, np.asarray(ref[key]))}
            err[p] = e
        res["err_vs_oracle"] = {"targets": int(sel.size), "sample_seed": ref.get("sample_seed"),
                                **err}
    if with_other:
        a, b = outs[precision], outs[other]
        refv = outs["fp64"]
        res["err_vs_fp64"] = {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(refv)),
                              "rel_max": float(np.abs(a - b).max() / np.abs(refv).max())}

    plan = plans[precision]
    call = caller(plan)
    # one counted call gives the work units; the timed calls count nothing
    plan.count_work(True)
    call()
    near_units, spread_units = plan.work()
    plan.count_work(False)
    stage = args.roofline_stage
    if stage == "auto":
        # the dominant of the two pair kernels, timed before the measured region
        per = {}
        for st in ("near", "spread"):
            _, per[st] = time_steps(plan, call, 5, 1, stage=st)
        stage = max(per, key=per.get)
    side = "spread" if stage == "near" else "near"
    ms, stage_ms = time_steps(plan, call, args.steps, args.warmup, stage=stage)
    _, side_ms = time_steps(plan, call, max(5, args.steps // 2), 2, stage=side)
    peak = PEAK_FP32_TFLOPS if precision == "mixed" else PEAK_FP64_TFLOPS
    flop_near = FLOP_NEAR_DL if dl else FLOP_NEAR_SL
    rl = {}
    for st, sms in ((stage, stage_ms), (side, side_ms)):
        units, flop = (near_units, flop_near) if st == "near" else (spread_units, FLOP_SPREAD)
        rl[st] = roofline_entry(st, sms, units, flop, peak, measured_traffic(st, c.name, precision))
    res["roofline_step"] = step_roofline(c, precision, dl, near_units, spread_units, ms)
    res.update(ms=ms, mpts=c.nt / (ms * 1e-3) / 1e6, stage=stage, roofline=rl[stage],
               roofline_other=rl[side], work={"near_pairs": near_units,
                                              "spread_updates": spread_units})
    if with_other:
        ms_o, _ = time_steps(plans[other], caller(plans[other]), max(5, args.steps // 2), 2)
        res[f"{other}_ms_per_step"] = round(ms_o, 5)
        res[f"{other}_mpoints_per_s"] = round(c.nt / (ms_o * 1e-3) / 1e6, 3)
        fp64_ms = ms_o if other == "fp64" else ms
        mixed_ms = ms if other == "fp64" else ms_o
        res["speedup_mixed_vs_fp64"] = round(fp64_ms / mixed_ms, 3)
    for p in plans.values():
        p.close()
    return res


def cheb_stage_rates(plan, call, c, steps):
    """HIP-event times of the forward and inverse Chebyshev stages and their
    achieved HBM rate: each reads and writes its fields once (FP32 complex
    half spectrum: Ny x 2 Nx (Nz/2 + 1) reals per field).  `call` evaluates
    the global part only, so no local sum shares the GPU with these stages."""
    dl = c.normals is not None
    per_field = c.Ny * 2 * c.Nx * (c.Nz // 2 + 1) * 4 * 2
    out = {}
    for st, nf in (("cheb_fwd", 3), ("cheb_inv", 6 if dl else 3)):
        _, ms = time_steps(plan, call, steps, 2, stage=st)
        out[st] = {"ms": round(ms, 5), "bytes": nf * per_field,
                   "GB_per_s": round(nf * per_field / (ms * 1e-3) / 1e9, 1)}
    return out


def measure_variant(c, args, precision):
    """Throughput, error against the stored oracle sample and Chebyshev stage
    rates of one more precision mode on the same workload."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G

    dev = torch.device("cuda:0")
    dl = c.normals is not None
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xs, f = t(c.xs), t(c.f)
    nrm = t(c.normals) if dl else None
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=dev)
    plan = G.Plan.from_case(c, precision=precision, sync_checks=False)

    def caller(parts=G.PART_ALL):
        if dl:
            return lambda: plan.double_layer(xs, f, xs, nrm, parts=parts, out=out)
        return lambda: plan.single_layer(xs, f, xs, parts=parts, out=out)

    res = {}
    ref = golden(c)
    if ref is not None:
        sel = np.asarray(ref["targets"])
        err = {}
        for key, parts in (("total", G.PART_ALL), ("local", G.PART_LOCAL),
                           ("global", G.PART_GLOBAL)):
            caller(parts)()
            plan.status()
            o = out.cpu().numpy()[sel]
            err[key] = {"rel_l2": rel_l2(o, np.asarray(ref[key])),
                        "rel_max": rel_max(o, np.asarray(ref[key]))}
        res["err_vs_oracle"] = err
    ms, _ = time_steps(plan, caller(), max(5, args.steps // 2), 2)
    res.update(ms_per_step=round(ms, 5), mpoints_per_s=round(c.nt / (ms * 1e-3) / 1e6, 3),
               chebyshev=cheb_stage_rates(plan, caller(G.PART_GLOBAL), c,
                                          max(5, args.steps // 2)))
    plan.close()
    return res


def extra_small(args):
    """64 forces + 1,000 probes: microseconds per call (latency-bound)."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    from workloads import case_small_sl

    c = case_small_sl(0)
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xs, f, xt = t(c.xs), t(c.f), t(c.xt)
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=dev)
    res = {"workload": c.name, "targets": c.nt, "sources": c.ns, "grid": [c.Nx, c.Nz, c.Ny]}
    ref = None
    for p in ("fp64", "mixed"):
        plan = G.Plan.from_case(c, precision=p, sync_checks=False)
        call = lambda: plan.single_layer(xs, f, xt, out=out)  # noqa: E731
        ms, _ = time_steps(plan, call, 200, 20)
        lat = []
        for _ in range(50):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e6)
        o = out.cpu().numpy()
        if p == "fp64":
            ref = o
        # the same call captured once into a HIP graph on a side stream and
        # replayed (one submission instead of about 30 launches)
        st = torch.cuda.Stream()
        plan.set_stream(st)
        with torch.cuda.stream(st):
            call()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=st):
            call()
        for _ in range(20):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(200):
            graph.replay()
        torch.cuda.synchronize()
        us_graph = (time.perf_counter() - t0) / 200 * 1e6
        plan.status()
        graph_err = float(np.abs(out.cpu().numpy() - o).max())
        res[p] = {"us_per_call_back_to_back": round(ms * 1e3, 2),
                  "us_per_call_synchronised_median": round(statistics.median(lat), 2),
                  "us_per_call_graph_replay": round(us_graph, 2),
                  "graph_replay_max_abs_diff": graph_err}
        if p == "mixed":
            res[p]["rel_l2_vs_fp64"] = rel_l2(o, ref)
        plan.close()
    return res


def extra_capsules_sl(args):
    from workloads import case_capsules_sl
    c = case_capsules_sl(1)
    r = measure_case(c, args, "mixed", with_other=True, golden_parts=False)
    return {"workload": c.name, "points": c.nt, "grid": [c.Nx, c.Nz, c.Ny],
            "mpoints_per_s": round(r["mpts"], 3), "ms_per_step": round(r["ms"], 5),
            "fp64_mpoints_per_s": r.get("fp64_mpoints_per_s"),
            "speedup_mixed_vs_fp64": r.get("speedup_mixed_vs_fp64"),
            "err_vs_fp64": r.get("err_vs_fp64"), "err_vs_oracle": r.get("err_vs_oracle"),
            "roofline": r["roofline"], "roofline_other": r["roofline_other"],
            "work": r["work"]}


def batched(args, steps):
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
    branches, tuned_ms, cached, cells = args.branches, None, None, None
    if branches <= 0:
        from paper_1109_6587_amd.autotune import tune_batch
        branches, tuned_ms, cached, cells = tune_batch(
            cases, (so, xs, f, to, xs, out[args.precision]), precision=args.precision, log=log)
    batches = {p: G.Batch(cases, precision=p, n_branches=branches,
                          cell_scales=cells if p == args.precision else None) for p in out}
    for p, b in batches.items():
        b.capture(so, xs, f, to, xs, out[p])
        b.replay()
        b.status()
    err = float(torch.linalg.norm(out["mixed"] - out["fp64"]) / torch.linalg.norm(out["fp64"]))

    def timed(b, k):
        for _ in range(args.warmup):
            b.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            b.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    prec = args.precision
    other = "fp64" if prec == "mixed" else "mixed"
    ms = timed(batches[prec], steps)
    ms_other = timed(batches[other], max(5, steps // 2))
    batches[prec].status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        batches[prec].single_layer(so, xs, f, to, xs, out[prec])
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / 5
    for b in batches.values():
        b.close()
    # roofline of the instances' pair kernels: every instance evaluated alone
    # (its own plan, one stream), kernel-counted work and event-timed stages
    # summed over the instances
    units = {"near": 0, "spread": 0}
    stage_ms = {"near": 0.0, "spread": 0.0}
    for i, c in enumerate(cases):
        plan = G.Plan.from_case(c, precision=prec, sync_checks=False,
                                cell_scale=cells[i] if cells else 0.0)
        xsi, fi = xs[so[i]:so[i + 1]], f[so[i]:so[i + 1]]
        oi = out[prec][to[i]:to[i + 1]]
        call = lambda: plan.single_layer(xsi, fi, xsi, out=oi)  # noqa: E731
        plan.count_work(True)
        call()
        nu, su = plan.work()
        plan.count_work(False)
        units["near"] += nu
        units["spread"] += su
        for st in ("near", "spread"):
            stage_ms[st] += time_steps(plan, call, 5, 1, stage=st)[1]
        plan.close()
    peak = PEAK_FP32_TFLOPS if prec == "mixed" else PEAK_FP64_TFLOPS
    rl = {st: roofline_entry(st, stage_ms[st], units[st],
                             FLOP_NEAR_SL if st == "near" else FLOP_SPREAD, peak, None)
          for st in ("near", "spread")}
    dom = max(stage_ms, key=stage_ms.get)
    for r in rl.values():
        r["scope"] = "sum over the 48 instances, each evaluated alone"
    return {"workload": "batched_48", "instances": len(cases), "points": n, "precision": prec,
            "roofline": rl[dom], "roofline_other": rl["spread" if dom == "near" else "near"],
            "branches": branches, "submission": "hip graph",
            "mpoints_per_s": round(n / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 5),
            f"{other}_ms_per_step": round(ms_other, 5), "eager_ms_per_step": round(ms_eager, 5),
            "err_vs_fp64": {"rel_l2": err},
            "autotune": {"ms_by_branches": tuned_ms, "from_cache": cached,
                         "cell_scales": cells}}


def fredholm(steps):
    """Seconds per Fredholm solve to 1e-6 on 100 drops in shear (64,200 nodes,
    192,600 unknowns, 384,000 Gauss-point sources): the drop run, training of
    the warm-start network on its first 3/4 and every start on the rest."""
    from paper_1109_6587_amd.warmstart import run
    from workloads import case_shear_drops
    train = (3 * steps) // 4
    res, _ = run(case_shear_drops(4), steps=steps, train_steps=train, log=log)
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
        # the fair baseline is the extrapolated start q_prev + dq_prev
        "speedup_learned_vs_extrapolated": round(res["speedup_vs_extrapolated"], 4),
        "products_saved_vs_extrapolated": round(res["products_saved_vs_extrapolated"], 3),
        "learned_beats_extrapolated": bool(st["learned_judged"]["products_mean"]
                                           < st["extrapolated"]["products_mean"]),
        "prediction_rel_err": round(res["prediction_rel_err_mean"], 4),
        "extrapolation_rel_err": round(res["extrapolation_rel_err_mean"], 4),
        "workload": res["workload"], "unknowns": res["unknowns"], "sources": res["sources"],
        "precision": res["precision"], "train_solves": res["train_solves"],
        "test_solves": res["test_solves"], "simulation_s": res["simulation_s"],
        "training_s": res["training_s"],
    }


def rigid_sphere():
    """The rigid-particle validation (workloads.case_rigid_sphere): the
    translational velocity at L = 3, 4, 5 wall spacings, its L^-2
    extrapolation beside the paper's 0.871, the GMRES products and seconds
    per solve, and the time of one boundary-integral single layer (element
    quadrature + global part, 2,562 nodes, 5,120 triangles, FP64)."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    from paper_1109_6587_amd.drops import incidence
    from workloads import case_rigid_sphere

    dev = torch.device("cuda:0")
    by_L = []
    for L in (3.0, 4.0, 5.0):
        c = case_rigid_sphere(L)
        off, adj = incidence(c.tri, len(c.nodes))
        ti = lambda a: torch.as_tensor(a, dtype=torch.int32, device=dev)  # noqa: E731
        m = (torch.as_tensor(c.nodes, dtype=torch.float64, device=dev), ti(c.tri), ti(off),
             ti(adj))
        plan = G.Plan(c.Lx, c.Lz, c.H, c.alpha, c.Nx, c.Nz, c.Ny, rc=c.rc, precision="fp64",
                      max_src=len(c.nodes), max_tgt=len(c.nodes))
        rp = G.RigidParticle(plan, len(c.nodes), len(c.tri), restart=100)
        uinf = G.poiseuille(plan, c.U0, m[0])
        f = torch.zeros_like(m[0])
        rp.single_layer(*m, uinf, out=f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            rp.single_layer(*m, uinf, out=f)
        torch.cuda.synchronize()
        prod_ms = (time.perf_counter() - t0) / 5 * 1e3
        f.zero_()
        t0 = time.perf_counter()
        U, W, iters, rel = rp.solve(*m, c.center, uinf, f, tol=1e-8, max_iter=800)
        solve_s = time.perf_counter() - t0
        log(f"rigid sphere L={L:g}: U/U0 {U[0]:.6f}, {iters} products, {solve_s:.3f} s")
        by_L.append({"L": L, "grid": [c.Nx, c.Nz, c.Ny], "U_over_U0": round(U[0], 6),
                     "Omega_max": max(abs(w) for w in W), "gmres_products": iters,
                     "rel_res": rel, "solve_s": round(solve_s, 4),
                     "single_layer_ms": round(prod_ms, 3)})
        rp.close()
        plan.close()
    Ls = np.array([r["L"] for r in by_L])
    c1, c0 = np.polyfit(Ls ** -2.0, np.array([r["U_over_U0"] for r in by_L]), 1)
    return {"workload": "rigid_sphere_5120", "nodes": 2562, "triangles": 5120,
            "extrapolated_U_over_U0": round(float(c0), 5), "paper_U_over_U0": 0.871,
            "by_L": by_L}


def spectral_eval(args):
    """The 50-capsule single layer with the global part evaluated off the mesh
    by its Fourier-Chebyshev series (Gaussian-gridding NUFFT in x, theta and
    z, msp = 6 mixed, 12 FP64) beside the 4th-order Lagrange stencil: ms per
    step, the event times of the evaluation kernel (interp stage) and of the
    deconvolution, oversampled inverse FFT and theta transform (fft_inv
    stage), and the error of each against the oracle's series at the stored
    sample of targets."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    from workloads import case_capsules_sl

    c = case_capsules_sl(1)
    dev = torch.device("cuda:0")
    xs = torch.as_tensor(c.xs, dtype=torch.float64, device=dev)
    f = torch.as_tensor(c.f, dtype=torch.float64, device=dev)
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=dev)
    ref = golden(c)
    want = sel = None
    path = os.path.join(ROOT, "tests", "golden", f"{c.name}_spectral_sampled.json")
    if ref is not None and os.path.exists(path):
        with open(path) as fh:
            spec = json.load(fh)
        if spec["targets"] == ref["targets"]:
            sel = np.asarray(ref["targets"])
            want = np.asarray(ref["local"]) + np.asarray(spec["global_spectral"])
    res = {"workload": c.name, "points": c.nt, "grid": [c.Nx, c.Nz, c.Ny],
           "oversampled_grid": [2 * c.Nx, 2 * c.Nz, c.Ny]}
    steps = max(5, args.steps // 2)
    for precision, msp in (("mixed", 6), ("fp64", 12)):
        plan = G.Plan.from_case(c, precision=precision, sync_checks=False)
        call = lambda: plan.single_layer(xs, f, xs, out=out)  # noqa: E731
        r = {"msp": msp}
        for mode, name in ((G.INTERP_LAGRANGE, "lagrange"), (G.INTERP_SPECTRAL, "spectral")):
            plan.set_interp(mode, msp)
            call()
            plan.status()
            e = {}
            if want is not None:
                o = out.cpu().numpy()[sel]
                e = {"rel_l2_vs_series": rel_l2(o, want), "rel_max_vs_series": rel_max(o, want)}
            ms, interp_ms = time_steps(plan, call, steps, 2, stage="interp")
            _, inv_ms = time_steps(plan, call, steps, 2, stage="fft_inv")
            r[name] = {"ms_per_step": round(ms, 5), "interp_ms": round(interp_ms, 5),
                       "fft_inv_ms": round(inv_ms, 5), **e}
        # window sums: one read and one FMA for each of the (2 msp)^3 window
        # nodes per field
        win = 3 * (2 * msp) ** 3 * c.nt
        r["window_reads_per_target"] = 3 * (2 * msp) ** 3
        r["window_fma_tflops"] = round(2 * win / (r["spectral"]["interp_ms"] * 1e-3) / 1e12, 3)
        res[precision] = r
        plan.close()
    return res


def probe_fields(args):
    """Velocity, pressure and stress at probes (ggem_probe): c0 (64 forces,
    1,000 probes; microseconds per call) and the 50-capsule forces of c1 at
    100,000 seeded probes (ms per call and probes per second), FP64 and
    mixed.  A call solves the global problem once for the stress (with the
    pressure gauge) and transforms the kept velocity and pressure
    coefficients back once more."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    from workloads import case_capsules_sl, case_small_sl

    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    res = {}
    c0 = case_small_sl(0)
    c1 = case_capsules_sl(1)
    rng = np.random.default_rng(17)
    npr = 100_000
    probes = np.stack([rng.uniform(0, c1.Lx, npr), rng.uniform(-c1.H, c1.H, npr),
                       rng.uniform(0, c1.Lz, npr)], 1)
    for name, c, xt in (("small_sl_64", c0, c0.xt), ("capsules_sl_50x642", c1, probes)):
        xs, f, xtd = t(c.xs), t(c.f), t(xt)
        nt = xt.shape[0]
        out = (torch.empty((nt, 3), dtype=torch.float64, device=dev),
               torch.empty((nt,), dtype=torch.float64, device=dev),
               torch.empty((nt, 6), dtype=torch.float64, device=dev))
        r = {"sources": c.ns, "probes": nt, "grid": [c.Nx, c.Nz, c.Ny]}
        for p in ("fp64", "mixed"):
            plan = G.Plan(c.Lx, c.Lz, c.H, c.alpha, c.Nx, c.Nz, c.Ny, rc=c.rc, precision=p,
                          max_src=c.ns, max_tgt=nt, sync_checks=False)
            call = lambda: plan.probe(xs, f, xtd, out=out)  # noqa: E731
            ms, _ = time_steps(plan, call, max(5, args.steps // 2), 2)
            r[p] = {"ms_per_call": round(ms, 4),
                    "mprobes_per_s": round(nt / (ms * 1e-3) / 1e6, 3)}
            plan.close()
        res[name] = r
    return res


def convergence_study():
    """The convergence experiment of Sec. 3.2.3 (Fig. ggem_conv) on the GPU,
    FP64: a point force (F, F, F) at (L/4, L/4, L/4) of a slit with
    L_x = L_z = wall spacing = L = 1, alpha = 80/3, observed at the mesh
    point (L/2, L/2, L/2) and at the off-mesh point (0.4312, 0.3734, 0.5234) L
    (the paper's frame, y from the lower wall), for r_c = C/alpha, C = 4, 5,
    6, and N_y from 17 to 129 with equal mean spacings (N_x = N_z = N_y - 1);
    relative error of u_x against N_y = 129 with r_c = 13/alpha (the paper's
    reference uses N_y = 225 and r_c = L/2; N_y is at most 129 here and r_c
    must stay below L/2), each off-mesh value with the Lagrange stencil and
    with the spectral evaluation (msp 12)."""
    import numpy as np
    import torch

    import paper_1109_6587_amd as G

    dev = torch.device("cuda:0")
    L, alpha = 1.0, 80.0 / 3.0
    H = 0.5 * L
    xs = torch.tensor([[0.25 * L, 0.25 * L - H, 0.25 * L]], dtype=torch.float64, device=dev)
    f = torch.ones((1, 3), dtype=torch.float64, device=dev)
    xt = torch.tensor([[0.5 * L, 0.5 * L - H, 0.5 * L], [0.4312 * L, 0.3734 * L - H, 0.5234 * L]],
                      dtype=torch.float64, device=dev)

    def ux(Ny, C, spectral):
        p = G.Plan(L, L, H, alpha, Ny - 1, Ny - 1, Ny, rc=C / alpha, precision="fp64",
                   max_src=1, max_tgt=2)
        if spectral:
            p.set_interp(G.INTERP_SPECTRAL, 12)
        u = p.single_layer(xs, f, xt).cpu().numpy()[:, 0]
        p.close()
        return u

    ref = ux(129, 13.0, True)
    rows = []
    for C in (4.0, 5.0, 6.0):
        for Ny in (17, 25, 33, 41, 49, 65, 81, 97, 121):
            ul, us = ux(Ny, C, False), ux(Ny, C, True)
            rows.append({"C": C, "Ny": Ny, "inv_alpha_dy": round((Ny - 1) / (alpha * L), 4),
                         "mesh_point": float(abs(ul[0] - ref[0]) / abs(ref[0])),
                         "off_mesh_lagrange": float(abs(ul[1] - ref[1]) / abs(ref[1])),
                         "off_mesh_spectral": float(abs(us[1] - ref[1]) / abs(ref[1]))})
    log("convergence study: " + ", ".join(f"C={r['C']:g} Ny={r['Ny']}: {r['mesh_point']:.1e}/"
                                          f"{r['off_mesh_lagrange']:.1e}/{r['off_mesh_spectral']:.1e}"
                                          for r in rows if r["Ny"] in (33, 121)))
    return {"workload": "point_force_convergence", "reference": {"Ny": 129, "C": 13.0,
                                                                 "u_x": [float(v) for v in ref]},
            "rows": rows}


def capsule_stages(steps=4):
    """The timing study of the capsule suspensions (Sec. 7.2, Fig. tscale):
    wall-clock ms per stage of the midpoint rule for 15, 30, 60 and 120
    neo-Hookean capsules of 320 triangles at volume fraction 0.15 and
    lambda = 1, 2, 5 (mixed precision, GMRES to the paper's relative
    residual 1e-4, warm started from the previous stage), after one warm-up
    step; with the GMRES products per solve, the adaptive time step, the
    volume corrections and the largest volume drift before correction."""
    import torch

    from paper_1109_6587_amd.capsules import CapsuleSuspension
    from workloads import case_capsule_suspension

    rows = []
    for lam in (1.0, 2.0, 5.0):
        for n in (15, 30, 60, 120):
            c = case_capsule_suspension(n, lam)
            sim = CapsuleSuspension(c, precision="mixed", tol=1e-4)
            sim.step()
            first = len(sim.stages)
            for _ in range(steps):
                sim.step()
            st = sim.stages[first:]
            solves = [r.iters for r in st]
            v = sim.membrane.volumes(sim.x)
            drift = float(torch.max(torch.abs(v / sim.v0 - 1.0)))
            row = {"capsules": n, "lambda": lam, "grid": [c.Nx, c.Nz, c.Ny],
                   "nodes": int(c.nodes.shape[0]), "triangles": int(c.tri.shape[0]),
                   "ms_per_stage": round(1e3 * statistics.median(r.seconds for r in st), 3),
                   "gmres_products_per_solve": round(statistics.mean(solves), 2),
                   "dt": round(sim.steps[-1].dt, 5),
                   "volume_corrections": sum(r.volume_corrections for r in sim.steps),
                   "overlap_sweeps": sum(r.overlap_sweeps for r in sim.steps),
                   "volume_drift_max": drift}
            log(f"capsules {n} lambda {lam:g}: {row['ms_per_stage']} ms/stage, "
                f"{row['gmres_products_per_solve']} products")
            rows.append(row)
            sim.close()
    return {"workload": "capsule_suspensions_320", "steps_timed": steps, "gmres_tol": 1e-4,
            "rows": rows, "volume_conservation": capsule_volume_drift()}


def capsule_volume_drift():
    """Volume conservation of one capsule in shear without correction (the
    check of Sec. 5: lambda = 5, Ca = 0.6, volume change over a unit
    strain): a pre-inflated 320-triangle capsule of radius 1 centred in an
    8 x 8 x 8 slit (grid 64 x 64 x 65, alpha = 4, r_c = 1), FP64, GMRES to
    1e-6, adaptive steps to gamma_dot t = 1; the relative volume change at
    the end and its largest magnitude on the way."""
    import numpy as np
    import torch

    from paper_1109_6587_amd.capsules import CapsuleSuspension
    from workloads import CapsuleCase, icosphere

    V, F = icosphere(2)
    cen = np.array([4.0, 0.0, 4.0])
    c = CapsuleCase("capsule_1x162_lam5", 8.0, 8.0, 4.0, 4.0, 1.0, 64, 64, 65, cen + V,
                    cen + V / 1.05, F.astype(np.int32), 1, len(V), 1.0, 5.0, 0.6, 1.0 / 0.6, 1.0,
                    0.05, {})
    sim = CapsuleSuspension(c, precision="fp64", tol=1e-6, vol_tol=np.inf)
    t, worst = 0.0, 0.0
    while t < 1.0 - 1e-12:
        h = sim.min_separation()
        t += sim.step(min(sim.time_step(h), 1.0 - t))
        d = float(sim.membrane.volumes(sim.x)[0] / sim.v0[0] - 1.0)
        worst = max(worst, abs(d))
    res = {"strain": round(t, 6), "steps": len(sim.steps), "relative_volume_change": d,
           "largest_relative_change": worst,
           "gmres_products_per_solve": round(statistics.mean(r.iters for r in sim.stages), 2),
           "paper": "about 1e-4 over a unit strain (lambda = 5, Ca = 0.6)"}
    log(f"capsule volume over a unit strain: {d:.2e} ({len(sim.steps)} steps)")
    sim.close()
    torch.cuda.synchronize()
    return res


def base_line(args, value, ms, dtype, config):
    return {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": config,
    }


def bench_single(args):
    from workloads import case_capsules_dl, case_capsules_sl

    c = case_capsules_sl(1) if args.workload == "capsules_sl" else case_capsules_dl(2)
    dl = c.normals is not None
    log(f"workload {c.name}: {c.nt} targets, grid {c.Nx}x{c.Nz}x{c.Ny}, {args.precision}")
    if args.serialized:
        return bench_serialized(args, c)
    r = measure_case(c, args, args.precision, with_other=not args.no_fp64)
    config = {"workload": c.name, "points": c.nt, "sources": c.ns,
              "grid": [c.Nx, c.Nz, c.Ny], "alpha": c.alpha, "rc": c.rc,
              "box": [c.Lx, 2 * c.H, c.Lz], "precision": args.precision,
              "layer": "double" if dl else "single"}
    line = base_line(args, r["mpts"], r["ms"], "f32+f64" if args.precision == "mixed" else "f64",
                     config)
    for k in ("err_vs_oracle", "err_vs_fp64", "fp64_ms_per_step", "fp64_mpoints_per_s",
              "mixed_ms_per_step", "mixed_mpoints_per_s", "speedup_mixed_vs_fp64", "work",
              "roofline_other", "roofline_step"):
        if k in r:
            line[k] = r[k]
    line["roofline"] = r["roofline"]
    if args.precision == "mixed":
        # the same workload with the Chebyshev transforms as BF16 hi + lo
        # split products (and the FP32-MFMA transforms' rates beside them)
        line["mixed_bf16"] = measure_variant(c, args, "mixed_bf16")
        line["mixed_chebyshev"] = measure_variant(c, args, "mixed")["chebyshev"]
    return c, line


def bench_serialized(args, c):
    import numpy as np
    import torch

    import paper_1109_6587_amd as G
    dev = torch.device("cuda:0")
    dl = c.normals is not None
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    xs, f = t(c.xs), t(c.f)
    nrm = t(c.normals) if dl else None
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=dev)
    plan = G.Plan.from_case(c, precision=args.precision, sync_checks=False)
    call = ((lambda: plan.double_layer(xs, f, xs, nrm, out=out)) if dl
            else (lambda: plan.single_layer(xs, f, xs, out=out)))
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
    line = base_line(args, c.nt / (ms * 1e-3) / 1e6, ms,
                     "f32+f64" if args.precision == "mixed" else "f64",
                     {"workload": c.name, "points": c.nt, "grid": [c.Nx, c.Nz, c.Ny],
                      "precision": args.precision, "mode": "serialized graph"})
    line["metric"] = "GGEM Mpoints/s, one evaluation per graph replay on a single stream"
    line["roofline"] = None
    return c, line


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built", file=sys.stderr)
        sys.exit(2)
    extras = [] if args.extras in ("", "none") else args.extras.split(",")
    for e in extras:
        if e not in EXTRAS:
            print(f"unknown extra workload {e!r}", file=sys.stderr)
            sys.exit(2)
    if args.workload == "extras":
        runs = {"small": ("small_sl_64", lambda: extra_small(args)),
                "capsules_sl": ("capsules_sl_50x642", lambda: extra_capsules_sl(args)),
                "batched": ("batched_48", lambda: batched(args, args.steps)),
                "fredholm": ("fredholm", lambda: fredholm(args.fredholm_steps)),
                "rigid": ("rigid_sphere", rigid_sphere),
                "spectral": ("spectral_eval", lambda: spectral_eval(args)),
                "capsules": ("capsule_stages", capsule_stages),
                "probes": ("probe_fields", lambda: probe_fields(args)),
                "convergence": ("convergence", convergence_study)}
        line = {"metric": "extra workloads only (no headline evaluation)", "n_gpus": 1}
        for e in extras:
            key, run = runs[e]
            log(f"extra: {key}")
            line[key] = run()
        print(json.dumps(line), flush=True)
        return
    if args.workload == "batched":
        r = batched(args, args.steps)
        line = base_line(args, r["mpoints_per_s"], r["ms_per_step"],
                         "f32+f64" if args.precision == "mixed" else "f64",
                         {"workload": "batched_48", "instances": r["instances"],
                          "points": r["points"], "precision": args.precision,
                          "branches": r["branches"], "submission": "hip graph"})
        line.update({k: v for k, v in r.items() if k not in line and k != "config"})
        line["roofline"] = r["roofline"]
        print(json.dumps(line), flush=True)
        return
    c, line = bench_single(args)
    if not args.serialized:
        if "small" in extras:
            log("extra: small_sl_64")
            line["small_sl_64"] = extra_small(args)
        if "capsules_sl" in extras:
            log("extra: capsules_sl_50x642")
            line["capsules_sl_50x642"] = extra_capsules_sl(args)
        if "batched" in extras:
            log("extra: batched_48")
            line["batched_48"] = batched(args, args.steps)
        if "fredholm" in extras:
            log("extra: fredholm")
            line["fredholm"] = fredholm(args.fredholm_steps)
        if "rigid" in extras:
            log("extra: rigid_sphere")
            line["rigid_sphere"] = rigid_sphere()
        if "spectral" in extras:
            log("extra: spectral evaluation")
            line["spectral_eval"] = spectral_eval(args)
        if "capsules" in extras:
            log("extra: capsule suspensions")
            line["capsule_stages"] = capsule_stages()
        if "probes" in extras:
            log("extra: probes")
            line["probe_fields"] = probe_fields(args)
        if "convergence" in extras:
            log("extra: convergence study")
            line["convergence"] = convergence_study()
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle)")
            line["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(line), flush=True)
    if args.calibrate_copy > 0:
        import torch
        n = args.calibrate_copy * (1 << 20)
        # known traffic for scaling the HBM counters: a fill (writes n bytes),
        # a device copy (reads and writes n) and a sum (reads n)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        tot = 0.0
        for _ in range(3):
            tot += float(src.view(torch.float32).sum())
        torch.cuda.synchronize()
        log(f"calibration: copied {n} bytes three times, summed them three times ({tot:.3e})")


if __name__ == "__main__":
    main()
