"""Expected values of the full-size parity tests, written by the FP64 oracle.

The two capsule workloads (50 capsules, 32,100 point forces, grid
128 x 128 x 65; 400 capsules, 1,536,000 Gauss-point forces, grid
256 x 256 x 65) are far too large for the oracle inside a test, so this
script evaluates it once at a fixed, seeded sample of targets and stores
the values as JSON beside itself.  It calls only the oracle and the input
generators.

    python tests/golden/make_fullsize.py sl    # ~2 minutes on 8 cores
    python tests/golden/make_fullsize.py dl    # about an hour

Each file records the workload, the sample indices and, per target, the
local part, the global part and their sum (single layer: velocity, Eq. u_g a;
double layer: traction n_k sigma_jk, Eq. wdbl).
"""
from __future__ import annotations

import json
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


def main(which):
    c = case_capsules_sl() if which == "sl" else case_capsules_dl()
    g = O.SlitGrid.from_case(c)
    sel = sample(c.xt.shape[0])
    t0 = time.time()
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
    main(sys.argv[1] if len(sys.argv) > 1 else "sl")
