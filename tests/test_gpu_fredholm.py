"""GMRES solve of the Fredholm equation (Eq. qa) through the C-ABI.

The library's operator equals the oracle's (FP64: 1e-10; mixed: 1e-5), and
the GMRES solution satisfies the ORACLE's equation to the requested tolerance
(a property check that holds at any size).
"""
import numpy as np
import pytest

import oracle as O
from workloads import case_small_surface

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def surf():
    c, tri, nrm, b = case_small_surface(5)
    return c, tri, nrm, b


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_fredholm_apply(surf, precision, tol):
    c, tri, nrm, b = surf
    print(f"fredholm apply {precision}", flush=True)
    g = O.SlitGrid.from_case(c)
    kappa = 2.0 / 3.0
    x = np.random.default_rng(1).standard_normal(b.shape)
    ref = O.fredholm_apply(g, c.xt, nrm, tri, kappa, x)
    plan = G.Plan.from_case(c, precision=precision, max_src=3 * tri.shape[0], max_tgt=c.nt)
    solver = G.FredholmSolver(plan, c.nt, tri.shape[0], restart=20)
    S = G.Surface(dev(c.xt), dev(nrm), dev(tri, torch.int32), kappa)
    y = solver.apply(S, dev(x)).cpu().numpy()
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_fredholm_solve(surf, precision, tol):
    c, tri, nrm, b = surf
    print(f"fredholm solve {precision}", flush=True)
    g = O.SlitGrid.from_case(c)
    kappa = 2.0 / 3.0
    plan = G.Plan.from_case(c, precision=precision, max_src=3 * tri.shape[0], max_tgt=c.nt)
    solver = G.FredholmSolver(plan, c.nt, tri.shape[0], restart=10)
    S = G.Surface(dev(c.xt), dev(nrm), dev(tri, torch.int32), kappa)
    q = torch.zeros((c.nt, 3), dtype=torch.float64, device=DEV)
    iters, rel = solver.solve(S, dev(b), q, tol=tol, max_iter=100)
    assert rel <= tol
    qn = q.cpu().numpy()
    res = np.linalg.norm(b - O.fredholm_apply(g, c.xt, nrm, tri, kappa, qn)) / np.linalg.norm(b)
    assert res < (3 * tol if precision == "fp64" else 5e-6)
    # a warm start at the solution needs no iteration
    iters2, rel2 = solver.solve(S, dev(b), q, tol=max(tol, 2 * rel), max_iter=100)
    assert iters2 == 0


def test_fredholm_nonconvergence_reported(surf):
    c, tri, nrm, b = surf
    plan = G.Plan.from_case(c, max_src=3 * tri.shape[0], max_tgt=c.nt)
    solver = G.FredholmSolver(plan, c.nt, tri.shape[0], restart=2)
    S = G.Surface(dev(c.xt), dev(nrm), dev(tri, torch.int32), 2.0 / 3.0)
    q = torch.zeros((c.nt, 3), dtype=torch.float64, device=DEV)
    iters, rel = solver.solve(S, dev(b), q, tol=1e-16, max_iter=2)
    assert iters == 2 and rel > 1e-16
