"""Expected values of the full-size parity tests, written by the FP64 oracle.

The two capsule workloads (50 capsules, 32,100 point forces, grid
128 x 128 x 65; 400 capsules, 1,536,000 Gauss-point forces, grid
256 x 256 x 65) are far too large for the oracle inside a test, so this
script evaluates it once at a fixed, seeded sample of targets and stores
the values as JSON beside itself.  It calls only the oracle and the input
generators.

    python tests/golden/make_fullsize.py sl      # ~2 minutes on 8 cores
    python tests/golden/make_fullsize.py dl 8    # wall data on 8 processes
    python tests/golden/make_fullsize.py sl_spectral

Each file records the workload, the sample indices and, per target, the
local part, the global part and their sum (single layer: velocity, Eq. u_g a;
double layer: traction n_k sigma_jk, Eq. wdbl).  ``sl_spectral`` writes the
single layer's global part at the same targets as the direct sum of its
Fourier-Chebyshev series (oracle/spectral.py), the reference of the
spectrally accurate off-mesh evaluation.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from workloads import case_capsules_dl, case_capsules_sl  # noqa: E402

NSAMPLE = 256
SAMPLE_SEED = 11


def sample(nt):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(nt, NSAMPLE, replace=False))


_W = {}


def _wall_chunk(rng):
    a, b = rng
    return O.local_velocity(_W["g"], _W["xs"], _W["f"], _W["pts"][a:b])


def parallel_wall_data(g, xs, f, workers):
    """The oracle's wall data with its local sum split over wall-node chunks.

    Every wall node's sum is formed by oracle.local_velocity over all sources
    in the same order whatever the chunk, so the values are bitwise those of
    oracle.wall_data; only the work is spread over processes.
    """
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    pts = np.concatenate([np.stack([X.ravel(), np.full(X.size, yw), Z.ravel()], axis=1)
                          for yw in (-g.H, g.H)])
    _W.update(g=g, xs=xs, f=f, pts=pts)
    step = 512
    chunks = [(a, min(a + step, len(pts))) for a in range(0, len(pts), step)]
    with mp.get_context("fork").Pool(workers) as pool:
        ul = np.concatenate(pool.map(_wall_chunk, chunks))
    n = X.size
    return -ul[:n].T.reshape(3, g.Nx, g.Nz), -ul[n:].T.reshape(3, g.Nx, g.Nz)


def main_spectral():
    import oracle.spectral as S
    c = case_capsules_sl()
    g = O.SlitGrid.from_case(c)
    sel = sample(c.xt.shape[0])
    t0 = time.time()
    xs = g.wrap(c.xs)
    coef = S.global_coefficients(g, xs, np.asarray(c.f, dtype=np.float64))
    print(f"coefficients done {time.time() - t0:.0f} s", flush=True)
    glo = S.evaluate(g, coef, g.wrap(c.xt[sel]))
    out = {
        "workload": c.name,
        "seed": int(c.meta["seed"]),
        "grid": [c.Nx, c.Nz, c.Ny],
        "sample_seed": SAMPLE_SEED,
        "targets": [int(i) for i in sel],
        "global_spectral": glo.tolist(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(HERE, f"{c.name}_spectral_sampled.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


def main(which, workers=1):
    if which == "sl_spectral":
        return main_spectral()
    c = case_capsules_sl() if which == "sl" else case_capsules_dl()
    g = O.SlitGrid.from_case(c)
    sel = sample(c.xt.shape[0])
    t0 = time.time()
    if workers > 1:
        # the global part calls oracle.ggem.wall_data(g, xs, f) with the wrapped
        # sources; hand it the same values computed in parallel
        xs_w = g.wrap(c.xs)
        f64 = np.asarray(c.f, dtype=np.float64)
        walls = parallel_wall_data(g, xs_w, f64, workers)
        print(f"wall data done {time.time() - t0:.0f} s", flush=True)

        def wall_data(g_, xs_, f_):
            assert g_ is g and np.array_equal(xs_, xs_w) and np.array_equal(f_, f64)
            return walls

        O.ggem.wall_data = wall_data
    if which == "sl":
        loc = O.single_layer(g, c.xs, c.f, c.xt[sel], parts=O.LOCAL)
        print(f"local done {time.time() - t0:.0f} s", flush=True)
        glo = O.single_layer(g, c.xs, c.f, c.xt[sel], parts=O.GLOBAL)
    else:
        loc = O.double_layer(g, c.xs, c.f, c.xt[sel], c.normals[sel], parts=O.LOCAL)
        print(f"local done {time.time() - t0:.0f} s", flush=True)
        glo = O.double_layer(g, c.xs, c.f, c.xt[sel], c.normals[sel], parts=O.GLOBAL)
    print(f"global done {time.time() - t0:.0f} s", flush=True)
    out = {
        "workload": c.name,
        "seed": int(c.meta["seed"]),
        "grid": [c.Nx, c.Nz, c.Ny],
        "sample_seed": SAMPLE_SEED,
        "targets": [int(i) for i in sel],
        "local": loc.tolist(),
        "global": glo.tolist(),
        "total": (loc + glo).tolist(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(HERE, f"{c.name}_sampled.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "sl", int(sys.argv[2]) if len(sys.argv) > 2 else 1)
