"""Autotuner for batched evaluations, with an on-disk cache.

The tunable of a batch is its number of branch streams: more branches let
small instances overlap, fewer keep large instances from competing for the
compute units.  For a batch (its instances' boxes, grids, split parameters
and point counts, the precision and the device name) every candidate is
timed as a captured graph (warm-up replays, then timed replays) and the
fastest is kept in a JSON cache, so later runs of the same batch shape skip
the search.  Cache file: $GGEM_AUTOTUNE_CACHE, else
~/.cache/ggem/autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import ggem as B

CANDIDATES = (1, 2, 4, 8)


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


def tune_batch(cases, arrays, precision="mixed", candidates=CANDIDATES, warmup=2, reps=5,
               path=None, log=None):
    """Best branch count for `cases`; arrays = (src_off, xs, f, tgt_off, xt, u)
    as for Batch.capture.  Returns (branches, timings in ms, from_cache)."""
    import torch
    path = path or cache_path()
    key = batch_key(cases, precision)
    data = _load(path)
    if key in data:
        ent = data[key]
        return int(ent["branches"]), ent.get("ms", {}), True
    times = {}
    for nb in candidates:
        b = B.Batch(cases, precision=precision, n_branches=nb)
        b.capture(*arrays)
        for _ in range(warmup):
            b.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.replay()
        torch.cuda.synchronize()
        times[str(nb)] = (time.perf_counter() - t0) * 1e3 / reps
        b.status()
        b.close()
        if log:
            log(f"branches {nb}: {times[str(nb)]:.3f} ms")
    best = int(min(times, key=times.get))
    data = _load(path)
    data[key] = {"branches": best, "ms": times, "instances": len(cases), "precision": precision}
    _store(path, data)
    return best, times, False
