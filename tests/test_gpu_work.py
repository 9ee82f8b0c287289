"""Work units counted by the kernels (ggem_plan_work) against brute-force
counts, and counting switched off by default (ggem_plan_count_work).

The counts are the work units of the benchmark's roofline figures: pairs
0 < |d| <= r_c of the local sum (Eq. u_loc, minimum image in x and z) and
(source, grid node) pairs within r_c of the global density (Eq. rho_l_g a).
The brute force here is plain numpy over all pairs, not the oracle.
"""
import numpy as np
import pytest

from workloads import random_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def min_image(d, L):
    return d - L * np.rint(d / L)


def brute_pairs(c):
    n = 0
    for a in range(0, c.xt.shape[0], 256):
        t = c.xt[a:a + 256]
        dx = min_image(t[:, None, 0] - c.xs[None, :, 0], c.Lx)
        dy = t[:, None, 1] - c.xs[None, :, 1]
        dz = min_image(t[:, None, 2] - c.xs[None, :, 2], c.Lz)
        r2 = (dx * dx + dy * dy) + dz * dz
        n += int(np.count_nonzero((r2 > 0) & (r2 <= c.rc * c.rc)))
    return n


def brute_updates(c):
    x = np.arange(c.Nx) * (c.Lx / c.Nx)
    z = np.arange(c.Nz) * (c.Lz / c.Nz)
    y = c.H * np.cos(np.pi * np.arange(c.Ny) / (c.Ny - 1))
    n = 0
    for s in c.xs:
        dx = min_image(x - s[0], c.Lx)
        dy = y - s[1]
        dz = min_image(z - s[2], c.Lz)
        r2 = (dx[None, :, None] ** 2 + dy[:, None, None] ** 2) + dz[None, None, :] ** 2
        n += int(np.count_nonzero(r2 <= c.rc * c.rc))
    return n


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("dl", [False, True])
def test_work_counts(precision, dl):
    # 6 x 6 cells across the periodic directions: the mixed local sum takes
    # its staged-image path
    c = random_case(41, 300, 200, 12.0, 2.0, 2.0, 2.0, 48, 48, 33, dl=dl)
    print(f"work counts {precision} dl={dl}", flush=True)
    plan = G.Plan.from_case(c, precision=precision)
    xs, f, xt = dev(c.xs), dev(c.f), dev(c.xt)
    out = torch.empty((c.nt, 3), dtype=torch.float64, device=DEV)

    def call():
        if dl:
            plan.double_layer(xs, f, xt, dev(c.normals), out=out)
        else:
            plan.single_layer(xs, f, xt, out=out)

    call()
    assert plan.work() == (0, 0)            # off by default
    ref = out.clone()
    plan.count_work(True)
    call()
    pairs, updates = plan.work()
    assert torch.equal(out, ref)           # counting does not change results
    plan.count_work(False)
    call()
    assert plan.work() == (0, 0)
    bp, bu = brute_pairs(c), brute_updates(c)
    print(pairs, bp, updates, bu, flush=True)
    if precision == "fp64":
        assert pairs == bp and updates == bu
    else:
        # FP32 cutoff decisions may differ for pairs within a rounding of r_c
        assert abs(pairs - bp) <= max(4, 1e-4 * bp)
        assert abs(updates - bu) <= max(4, 1e-4 * bu)
    plan.close()
