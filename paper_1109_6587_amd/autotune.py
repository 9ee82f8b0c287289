"""Autotuner for batched evaluations, with an on-disk cache.

A batch has two tunables.
* The cell size of each instance (ggem_params.cell_scale: cells of at least
  scale * r_c on a side).  Larger cells mean fewer, fuller cell rows for the
  spread and the local sum to walk, which helps sparse instances; smaller
  cells cull more candidate pairs, which helps dense ones.  Each instance is
  timed alone at every candidate scale and keeps its fastest.
* The number of branch streams: more branches let small instances overlap,
  fewer keep large instances from competing for the compute units.  Every
  candidate is timed as a captured graph of the whole batch (warm-up
  replays, then timed replays), with the tuned cell sizes.
The result for a batch shape (its instances' boxes, grids, split parameters
and point counts, the precision and the device name) is kept in a JSON
cache, so later runs of the same batch shape skip the search.  Cache file:
$GGEM_AUTOTUNE_CACHE, else ~/.cache/ggem/autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import ggem as B

CANDIDATES = (1, 2, 4, 8)
CELL_SCALES = (0.0, 1.5, 2.0)


def cache_path():
    return os.environ.get("GGEM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ggem", "autotune.json"))


def device_name():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def batch_key(cases, precision, device=None):
    desc = [precision, device if device is not None else device_name()]
    for c in cases:
        desc.append([round(float(v), 9) for v in (c.Lx, c.Lz, c.H, c.alpha, c.rc)]
                    + [int(c.Nx), int(c.Nz), int(c.Ny), int(c.ns), int(c.nt)])
    return hashlib.sha256(json.dumps(desc).encode()).hexdigest()[:32]


def _load(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(call, warmup, reps):
    import torch
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune_cells(cases, arrays, precision="mixed", scales=CELL_SCALES, warmup=2, reps=5):
    """Fastest cell scale of each instance, each evaluated alone (its own
    plan, eager calls); returns (scales, ms per instance and scale)."""
    so, xs, f, to, xt, u = arrays
    best, ms = [], []
    for i, c in enumerate(cases):
        a, b = int(so[i]), int(so[i + 1])
        p, q = int(to[i]), int(to[i + 1])
        xsi, fi, ui = xs[a:b], f[a:b], u[p:q]
        xti = xsi if (xt is xs and a == p and b == q) else xt[p:q]
        row = {}
        for sc in scales:
            plan = B.Plan.from_case(c, precision=precision, sync_checks=False, cell_scale=sc)
            row[str(sc)] = _time(lambda: plan.single_layer(xsi, fi, xti, out=ui), warmup, reps)
            plan.status()
            plan.close()
        ms.append(row)
        best.append(float(min(row, key=row.get)))
    return best, ms


def tune_batch(cases, arrays, precision="mixed", candidates=CANDIDATES, warmup=2, reps=5,
               path=None, log=None, scales=CELL_SCALES):
    """Best cell scales and branch count for `cases`; arrays = (src_off, xs,
    f, tgt_off, xt, u) as for Batch.capture.  Returns (branches, timings in
    ms by branch count, from_cache, cell scale per instance)."""
    path = path or cache_path()
    key = batch_key(cases, precision)
    data = _load(path)
    if key in data and "cell_scales" in data[key]:
        ent = data[key]
        return int(ent["branches"]), ent.get("ms", {}), True, [float(v) for v in ent["cell_scales"]]
    cells, cell_ms = tune_cells(cases, arrays, precision, scales, warmup, reps)
    if log:
        log(f"cell scales: {cells}")
    times = {}
    for nb in candidates:
        b = B.Batch(cases, precision=precision, n_branches=nb, cell_scales=cells)
        b.capture(*arrays)
        times[str(nb)] = _time(b.replay, warmup, reps)
        b.status()
        b.close()
        if log:
            log(f"branches {nb}: {times[str(nb)]:.3f} ms")
    best = int(min(times, key=times.get))
    data = _load(path)
    data[key] = {"branches": best, "ms": times, "instances": len(cases), "precision": precision,
                 "cell_scales": cells, "cell_ms": cell_ms}
    _store(path, data)
    return best, times, False, cells
