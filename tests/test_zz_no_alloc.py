"""The allocation-free single layer (ggem_single_layer_noalloc) against the
plan entry point ggem_single_layer, through the C ABI.

Two calls in a row share the library's static workspace; the second has
fewer sources and targets than the first (same parameters, so the constants
are not recomputed and the second call must not see the first call's
contents).  FP64 must match the plan path to 1e-10 (relative max-norm),
mixed precision to 1e-5 (relative 2-norm).  A workspace larger than the
static array is refused with GGEM_E_CAPACITY before any device work.
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
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def plan_result(c, ns, nt, precision, max_src, max_tgt):
    plan = G.Plan.from_case(c, precision=precision, max_src=max_src, max_tgt=max_tgt)
    u = plan.single_layer(dev(c.xs[:ns]), dev(c.f[:ns]), dev(c.xt[:nt]))
    out = u.cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_plan_two_calls(precision):
    c = random_case(31, 400, 300, 10.0, 1.0, 4.0, 1.0, 32, 32, 33)
    ns0, nt0 = c.ns, c.nt            # 400 sources, 700 targets
    sizes = [(ns0, nt0), (251, 333)]  # second call smaller than the first
    for k, (ns, nt) in enumerate(sizes):
        print(f"noalloc {precision} call {k}: ns={ns} nt={nt}", flush=True)
        u = G.single_layer_noalloc(c.Lx, c.Lz, c.H, c.alpha, c.Nx, c.Nz, c.Ny,
                                   dev(c.xs[:ns]), dev(c.f[:ns]), dev(c.xt[:nt]), rc=c.rc,
                                   precision=precision, max_src=ns0, max_tgt=nt0)
        torch.cuda.synchronize()
        got = u.cpu().numpy()
        ref = plan_result(c, ns, nt, precision, ns0, nt0)
        assert got.shape == (nt, 3)
        if precision == "fp64":
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
            assert err < 1e-10, err
        else:
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            assert err < 1e-5, err


def test_noalloc_rejects_oversized_workspace():
    c = random_case(32, 64, 16, 40.0, 6.0, 2.0, 2.0, 256, 256, 65)
    with pytest.raises(G.GGEMError) as e:
        G.single_layer_noalloc(c.Lx, c.Lz, c.H, c.alpha, c.Nx, c.Nz, c.Ny, dev(c.xs),
                               dev(c.f), dev(c.xt), rc=c.rc, precision="mixed")
    assert e.value.code == -3
