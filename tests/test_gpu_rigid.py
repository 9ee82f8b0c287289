"""Boundary-integral single layer on a triangulated surface and the rigid
particle (Sec. 3.4, Sec. 6.1) through the C-ABI, against oracle/bi.py, and
the paper's validation: a sphere between the walls in pressure-driven flow.
"""
import numpy as np
import pytest

import oracle as O
import oracle.bi as bi
from workloads.inputs import case_rigid_sphere, icosphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402
from paper_1109_6587_amd.drops import incidence  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def mesh(level, a, center):
    V, F = icosphere(level)
    nodes = V * a + np.asarray(center)
    off, adj = incidence(F, len(nodes))
    return nodes, F, (dev(nodes), dev(F, torch.int32), dev(off, torch.int32),
                      dev(adj, torch.int32))


def small_grid():
    return O.SlitGrid(2.0, 2.0, 0.75, 8.0, 0.5, 32, 32, 33)


_REF = {}


def reference(kind, center):
    """Oracle value of one layer on the level-2 sphere at `center` (cached:
    the same for both precisions)."""
    key = (kind, center)
    if key not in _REF:
        g = small_grid()
        V, F = icosphere(2)
        nodes = V * 0.3 + np.asarray(center)
        if kind == "sl":
            f = np.random.default_rng(11).standard_normal(nodes.shape)
            _REF[key] = (f, None, bi.sl_bi(g, nodes, F, f))
        else:
            nrm = O.node_normals(nodes, F)
            q = np.random.default_rng(12).standard_normal(nodes.shape)
            _REF[key] = (q, nrm, bi.dl_bi(g, nodes, F, nrm, q))
    return _REF[key]


def make(g, n, ntri, precision="fp64", restart=60):
    plan = G.Plan(g.Lx, g.Lz, g.H, g.alpha, g.Nx, g.Nz, g.Ny, rc=g.rc, precision=precision,
                  max_src=n, max_tgt=n)
    return plan, G.RigidParticle(plan, n, ntri, restart=restart)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
@pytest.mark.parametrize("center", [(1.0, 0.05, 1.0), (0.12, -0.1, 1.93)])
def test_bi_single_layer(precision, tol, center):
    """The element-quadrature local part and the nodal-trapezoid global part
    against the oracle, on a sphere inside the box and on one that crosses
    the periodic boundaries (unwrapped node positions)."""
    print(f"bi single layer {precision} {center}", flush=True)
    g = small_grid()
    nodes, F, m = mesh(2, 0.3, center)
    f, _, ref = reference("sl", center)
    plan, rp = make(g, len(nodes), len(F), precision)
    u = rp.single_layer(*m, dev(f)).cpu().numpy()
    assert np.abs(u - ref).max() < tol * np.abs(ref).max()
    rp.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
@pytest.mark.parametrize("center", [(1.0, 0.05, 1.0), (0.12, -0.1, 1.93)])
def test_bi_double_layer(precision, tol, center):
    """The element double layer with n~ on the elements at the target, and
    the stress of the nodal point forces, against the oracle."""
    print(f"bi double layer {precision} {center}", flush=True)
    g = small_grid()
    nodes, F, m = mesh(2, 0.3, center)
    q, nrm, ref = reference("dl", center)
    plan, rp = make(g, len(nodes), len(F), precision)
    v = rp.double_layer(*m, dev(nrm), dev(q)).cpu().numpy()
    assert np.abs(v - ref).max() < tol * np.abs(ref).max()
    rp.close()


def test_rigid_solve_matches_oracle():
    """GMRES on the GPU against the oracle's dense LU of the same system."""
    print("rigid solve vs oracle", flush=True)
    g = small_grid()
    xc = np.array([1.0, 0.0, 1.0])
    nodes, F, m = mesh(1, 0.3, xc)
    uinf_ref = bi.poiseuille(nodes, 1.0, g.H)
    f_ref, U_ref, W_ref = bi.rigid_solve(g, nodes, F, xc, uinf_ref)
    plan, rp = make(g, len(nodes), len(F))
    uinf = G.poiseuille(plan, 1.0, m[0])
    assert np.abs(uinf.cpu().numpy() - uinf_ref).max() < 1e-15
    f = torch.zeros_like(m[0])
    U, W, iters, rel = rp.solve(*m, xc, uinf, f, tol=1e-12, max_iter=400)
    print(U, W, iters, rel, U_ref, W_ref, flush=True)
    assert rel <= 1e-12
    assert np.abs(np.array(U) - U_ref).max() < 1e-9
    assert np.abs(np.array(W) - W_ref).max() < 1e-9
    fn = f.cpu().numpy()
    assert np.abs(fn - f_ref).max() < 1e-8 * np.abs(f_ref).max()
    rp.close()


def test_rigid_errors():
    g = small_grid()
    nodes, F, m = mesh(1, 0.3, (1.0, 0.0, 1.0))
    plan, rp = make(g, len(nodes), len(F))
    f = torch.zeros_like(m[0])
    bad = m[3].clone()
    bad[0] = (bad[0] + 7) % len(F)          # a triangle that does not hold node 0
    with pytest.raises(G.GGEMError):
        rp.single_layer(m[0], m[1], m[2], bad, f)
    small = G.RigidParticle(plan, len(nodes) - 1, len(F))
    with pytest.raises(G.GGEMError) as e:
        small.single_layer(*m, f)
    assert e.value.code == G.ggem.E_CAPACITY
    with pytest.raises(G.GGEMError):
        rp.solve(*m, (1.0, 0.0, 1.0), f, f, tol=0.0)
    small.close()
    rp.close()


def sphere_velocity(L, level=4):
    """Translational velocity of the force- and torque-free sphere of the
    rigid-particle validation (workloads.case_rigid_sphere)."""
    c = case_rigid_sphere(L, level)
    off, adj = incidence(c.tri, len(c.nodes))
    m = (dev(c.nodes), dev(c.tri, torch.int32), dev(off, torch.int32), dev(adj, torch.int32))
    plan = G.Plan(c.Lx, c.Lz, c.H, c.alpha, c.Nx, c.Nz, c.Ny, rc=c.rc, precision="fp64",
                  max_src=len(c.nodes), max_tgt=len(c.nodes))
    rp = G.RigidParticle(plan, len(c.nodes), len(c.tri), restart=100)
    uinf = G.poiseuille(plan, c.U0, m[0])
    f = torch.zeros_like(m[0])
    U, W, iters, rel = rp.solve(*m, c.center, uinf, f, tol=1e-8, max_iter=800)
    rp.close()
    plan.close()
    return U, W, iters, rel


def test_rigid_sphere_in_poiseuille_flow():
    """The paper's validation (Sec. 6.1): the velocity at L = 3, 4, 5 (in
    units of the wall spacing), extrapolated in L^-2 to an infinite slit,
    is 0.871 of the centre-line velocity (the paper's value, three digits)."""
    Ls = (3.0, 4.0, 5.0)
    Us = []
    for L in Ls:
        print(f"rigid sphere L={L}", flush=True)
        U, W, iters, rel = sphere_velocity(L)
        print(L, U, W, iters, rel, flush=True)
        assert rel <= 1e-8
        assert abs(U[1]) < 1e-4 and abs(U[2]) < 1e-4 and max(abs(w) for w in W) < 1e-4
        Us.append(U[0])
    c = np.polyfit(np.array(Ls) ** -2.0, np.array(Us), 1)
    print("U(L) =", Us, "extrapolated", c[1], flush=True)
    assert abs(c[1] - 0.871) < 0.005
