"""Neo-Hookean capsules through the C-ABI against oracle/capsule.py: membrane
traction jump and energy, volumes and the volume correction, separation and
the overlap correction, the right-hand side of Eq. qa, and whole midpoint
steps of a small suspension against the oracle's (Sec. 4, 5, 7.1)."""
import numpy as np
import pytest

import oracle as O
import oracle.bi as BI
import oracle.capsule as C
from oracle.surface import node_normals, surface_velocity
from workloads.inputs import CapsuleCase, icosphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402
from paper_1109_6587_amd.capsules import CapsuleSuspension  # noqa: E402
from paper_1109_6587_amd.drops import incidence  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def capsules(level, centres, radius, seed, amp):
    V, F = icosphere(level)
    rng = np.random.default_rng(seed)
    ref = np.concatenate([c + radius / 1.05 * V for c in centres])
    x = np.concatenate([c + radius * V for c in centres]) + amp * rng.standard_normal(ref.shape)
    tri = np.concatenate([F + k * len(V) for k in range(len(centres))]).astype(np.int32)
    return ref, x, tri


class Setup:
    def __init__(self, ref, x, tri, ncap, Gs=2.0, L=8.0, H=2.0):
        n, m = len(x), len(tri)
        self.plan = G.Plan(L, L, H, 4.0, 32, 32, 33, rc=1.0, max_src=3 * m, max_tgt=n)
        self.solver = G.FredholmSolver(self.plan, n, m)
        off, adj = incidence(tri, n)
        self.tri, self.off, self.adj = dev(tri, torch.int32), dev(off, torch.int32), dev(adj, torch.int32)
        self.mem = G.Membrane(self.solver, ncap, self.tri, dev(ref), Gs)

    def close(self):
        self.mem.close()
        self.solver.close()
        self.plan.close()


def test_membrane_traction_and_energy():
    cen = [np.array([1.0, 0.0, 1.0]), np.array([4.0, 0.3, 2.0]), np.array([6.5, -0.4, 5.0])]
    ref, x, tri = capsules(2, cen, 0.9, 1, 0.05)
    s = Setup(ref, x, tri, 3, Gs=1.7)
    df, e = s.mem.traction(dev(x), s.off, s.adj, energy=True)
    want, we = C.membrane_traction(ref, x, tri, 1.7)
    assert np.abs(df.cpu().numpy() - want).max() < 1e-12 * np.abs(want).max()
    assert abs(e - we) < 1e-12 * we
    # the reference state carries nothing
    z = s.mem.traction(dev(ref), s.off, s.adj).cpu().numpy()
    assert np.abs(z).max() < 1e-12
    s.close()


def test_membrane_errors():
    ref, x, tri = capsules(1, [np.zeros(3) + 1.0, np.array([4.0, 0, 4.0])], 0.9, 2, 0.0)
    n, m = len(x), len(tri)
    plan = G.Plan(8.0, 8.0, 2.0, 4.0, 32, 32, 33, rc=1.0, max_src=3 * m, max_tgt=n)
    solver = G.FredholmSolver(plan, n, m)
    bad = tri.copy()
    bad[3, 1] = n - 1                  # a node of the other capsule
    with pytest.raises(G.GGEMError) as e:
        G.Membrane(solver, 2, dev(bad, torch.int32), dev(ref), 1.0)
    assert e.value.code == G.ggem.E_ARG
    with pytest.raises(G.GGEMError):
        G.Membrane(solver, 2, dev(tri, torch.int32), dev(ref), 0.0)
    mem = G.Membrane(solver, 2, dev(tri, torch.int32), dev(ref), 1.0)
    off, adj = incidence(tri, n)
    adj = adj.copy()
    adj[5] = (adj[5] + 7) % m           # a triangle that does not hold the node
    with pytest.raises(G.GGEMError) as e:
        mem.traction(dev(x), dev(off, torch.int32), dev(adj, torch.int32))
    assert e.value.code == G.ggem.E_ARG
    mem.close()
    solver.close()
    plan.close()


def test_volumes_and_volume_correction():
    cen = [np.array([1.0, 0.0, 1.0]), np.array([4.0, 0.3, 2.0])]
    ref, x, tri = capsules(2, cen, 0.9, 3, 0.0)
    x[len(x) // 2:] = 1.01 * (x[len(x) // 2:] - cen[1]) + cen[1]
    s = Setup(ref, x, tri, 2)
    xd = dev(x)
    v = s.mem.volumes(xd).cpu().numpy()
    assert np.abs(v - C.volumes(x, tri, 2)).max() < 1e-13 * v.max()
    v0 = C.volumes(np.concatenate([c + 0.9 * icosphere(2)[0] for c in cen]), tri, 2)
    nrm, area, _ = s.solver.geometry(xd, s.tri, s.off, s.adj)
    k = s.mem.volume_correct(xd, nrm, area, dev(v0), 1e-4)
    want, moved = C.volume_correct(x, tri, node_normals(x, tri), 2, v0, 1e-4)
    assert k == int(moved.sum()) == 1
    assert np.abs(xd.cpu().numpy() - want).max() < 1e-13 * np.abs(want).max()
    s.close()


def test_separation_and_overlap_correction():
    V, F = icosphere(1)
    L, H, hm = 10.0, 3.0, 0.05
    cen = [[5.0, 0, 5.0], [6.9, 0.2, 5.1], [0.5, 0, 9.6], [9.5, 0.1, 9.7], [2.0, H - 1.01, 2.0]]
    x = np.concatenate([np.array(c) + V for c in cen])
    tri = np.concatenate([F + k * len(V) for k in range(5)]).astype(np.int32)
    s = Setup(x, x, tri, 5, L=L, H=H)
    xd = dev(x)
    e, g = s.mem.separation(xd, L, L, 1.0)
    gw = C.gaps(x, 5, L, L)
    assert abs(e - C.min_edge(x, tri)) < 1e-14
    assert abs(g - gw.min()) < 1e-14
    sweeps = s.mem.overlap_correct(xd, L, L, H, hm)
    want, ws = C.overlap_correct(x, 5, L, L, H, hm)
    assert sweeps == ws >= 1
    assert np.abs(xd.cpu().numpy() - want).max() < 1e-12
    # pairs farther apart than reach are reported as infinitely far
    _, g2 = s.mem.separation(xd, L, L, 0.01)
    assert g2 == np.inf
    s.close()


def test_traction_rhs():
    V, F = icosphere(2)
    x = V + [1.0, 0.0, 1.0]
    s = Setup(x, x, F.astype(np.int32), 1)
    rng = np.random.default_rng(7)
    df = rng.standard_normal(x.shape)
    n = node_normals(x, F)
    b = s.solver.traction_rhs(dev(n), dev(df), 3.0, 0.7).cpu().numpy()
    want = C.traction_rhs(n, df, 3.0, 0.7)
    assert np.abs(b - want).max() < 1e-15 * np.abs(want).max()
    s.close()


def small_case(lam):
    """Two level-1 capsules of radius 0.5 (stress-free radius 0.5/1.05,
    perturbed), L = 3, H = 1, grid 32 x 32 x 33, alpha = 4, r_c = 1."""
    ref, x, tri = capsules(1, [np.array([0.8, -0.3, 1.0]), np.array([2.1, 0.35, 1.8])], 0.5, 5, 0.01)
    return CapsuleCase("small", 3.0, 3.0, 1.0, 4.0, 1.0, 32, 32, 33, x, ref, tri, 2, 42, 0.5,
                       lam, 0.5, 2.0, 1.0, 0.025, {})


def oracle_velocity(c, g, x, q, disc):
    """u of Eq. bi_ua: the paper's element discretisation (u_inf + 8 pi times
    the discretised single layer) or the Gauss-point one."""
    if disc == "gauss":
        return surface_velocity(g, x, c.tri, q, c.shear)
    u = 8.0 * np.pi * BI.sl_bi(g, x, c.tri, q)
    u[:, 0] += c.shear * x[:, 1]
    return u


def oracle_stage(c, g, x, disc):
    nrm = node_normals(x, c.tri)
    df, _ = C.membrane_traction(c.ref_nodes, x, c.tri, c.G)
    b = C.traction_rhs(nrm, df, c.lam, c.shear)
    return oracle_velocity(c, g, x, b, disc)


@pytest.mark.parametrize("disc", ["bi", "gauss"])
def test_capsule_step_matches_the_oracle(disc):
    """One midpoint step of the matched-viscosity suspension (q = b), FP64,
    with the oracle's dt rule, against the oracle's step."""
    c = small_case(1.0)
    sim = CapsuleSuspension(c, precision="fp64", discretisation=disc)
    g = O.SlitGrid(c.Lx, c.Lz, c.H, c.alpha, c.rc, c.Nx, c.Nz, c.Ny)
    h = C.min_separation(c.nodes, c.tri, 2, c.Lx, c.Lz)
    assert abs(sim.min_separation() - h) < 1e-14
    dt = sim.step()
    assert abs(dt - C.time_step(h, c.ca, c.a, c.shear)) < 1e-15
    x = c.nodes
    u1 = oracle_stage(c, g, x, disc)
    u2 = oracle_stage(c, g, x + 0.5 * dt * u1, disc)
    x1 = x + dt * u2
    # the coarse, perturbed meshes drift by about 4e-3 in one step, so the
    # volume correction acts on both capsules; no overlap is corrected
    want, moved = C.volume_correct(x1, c.tri, node_normals(x1, c.tri), 2,
                                   C.volumes(x, c.tri, 2), 1e-4)
    got = sim.x.cpu().numpy()
    assert sim.steps[0].volume_corrections == int(moved.sum()) == 2
    assert sim.steps[0].overlap_sweeps == 0
    assert np.abs(got - want).max() < 1e-10 * np.abs(dt * u2).max()
    sim.close()


@pytest.mark.parametrize("disc", ["bi", "gauss"])
def test_capsule_stage_with_viscosity_contrast(disc):
    """lambda = 3: the GMRES density satisfies the oracle's Eq. qa and the
    velocity is the oracle's for that density."""
    c = small_case(3.0)
    sim = CapsuleSuspension(c, precision="fp64", tol=1e-10, discretisation=disc)
    u, q = sim.stage(sim.x, sim.q, 0)
    x = c.nodes
    nrm = node_normals(x, c.tri)
    df, _ = C.membrane_traction(c.ref_nodes, x, c.tri, c.G)
    b = C.traction_rhs(nrm, df, c.lam, c.shear)
    g = O.SlitGrid(c.Lx, c.Lz, c.H, c.alpha, c.rc, c.Nx, c.Nz, c.Ny)
    qn = q.cpu().numpy()
    kappa = (c.lam - 1) / (c.lam + 1)
    if disc == "gauss":
        r = O.fredholm_apply(g, x, nrm, c.tri, kappa, qn) - b
    else:
        r = qn + 2.0 * kappa * BI.dl_bi(g, x, c.tri, nrm, qn) - b
    assert np.abs(r).max() < 1e-8 * np.abs(b).max()
    want = oracle_velocity(c, g, x, qn, disc)
    assert np.abs(u.cpu().numpy() - want).max() < 1e-10 * np.abs(want).max()
    assert sim.stages[0].iters > 1
    sim.close()


def test_capsule_at_rest_stays_at_rest():
    """A pre-inflated capsule in quiescent fluid carries an isotropic tension
    whose traction drives (almost) no flow: its nodes move far less than
    the membrane's own velocity scale tau/mu over one step."""
    V, F = icosphere(2)
    c = CapsuleCase("rest", 4.0, 4.0, 1.5, 4.0, 1.0, 32, 32, 33, V + [2.0, 0, 2.0],
                    V / 1.05 + [2.0, 0, 2.0], F.astype(np.int32), 1, len(V), 1.0, 2.0, 0.5,
                    2.0, 0.0, 0.05, {})
    sim = CapsuleSuspension(c, precision="fp64", tol=1e-10)
    u, _ = sim.stage(sim.x, sim.q, 0)
    tau = c.G * (1 - 1.05 ** -6)
    assert np.abs(u.cpu().numpy()).max() < 2e-2 * tau
    sim.close()


def test_capsule_edge_cases():
    """A single capsule (no pairs), zero sweeps, a zero volume tolerance."""
    V, F = icosphere(1)
    x = V + [2.0, 0.0, 2.0]
    s = Setup(x, x, F.astype(np.int32), 1, L=8.0, H=2.0)
    xd = dev(x)
    e, g = s.mem.separation(xd, 8.0, 8.0, 1.0)
    assert abs(e - C.min_edge(x, F)) < 1e-14 and g == np.inf
    near_wall = dev(V + [2.0, 1.0, 2.0])          # 1.0 from y = +2 minus the radius 1: gap 0
    assert s.mem.overlap_correct(near_wall, 8.0, 8.0, 2.0, 0.05, max_sweeps=0) == 0
    assert torch.equal(near_wall, dev(V + [2.0, 1.0, 2.0]))
    assert s.mem.overlap_correct(near_wall, 8.0, 8.0, 2.0, 0.05) == 1
    assert abs(near_wall[:, 1].max().item() - (2.0 - 0.05)) < 1e-14
    nrm, area, _ = s.solver.geometry(xd, s.tri, s.off, s.adj)
    v0 = s.mem.volumes(xd) * (1 + 1e-9)
    assert s.mem.volume_correct(xd, nrm, area, v0, 0.0) == 1
    assert s.mem.volume_correct(xd, nrm, area, s.mem.volumes(xd).clone(), 0.0) == 0
    s.close()


def test_capsule_entry_point_errors():
    V, F = icosphere(1)
    x = V + [2.0, 0.0, 2.0]
    s = Setup(x, x, F.astype(np.int32), 1, L=8.0, H=2.0)
    xd = dev(x)
    nrm = dev(node_normals(x, F))
    rp = G.RigidParticle(s.plan, len(x), len(F))
    cases = [
        lambda: s.solver.traction_rhs(nrm, nrm, 0.0, 1.0),                 # lambda <= 0
        lambda: s.solver.traction_rhs(nrm, nrm, 2.0, float("nan")),        # shear not finite
        lambda: s.mem.separation(xd, 8.0, 8.0, 0.0),                       # reach <= 0
        lambda: s.mem.overlap_correct(xd, 8.0, 8.0, 2.0, 0.0),             # h_min <= 0
        lambda: s.mem.overlap_correct(xd, 8.0, 0.0, 2.0, 0.05),            # bad box
        lambda: rp.surface_velocity(xd, s.tri, s.off, s.adj, nrm, float("inf")),
        lambda: rp.fredholm_solve(xd, s.tri, s.off, s.adj, nrm, 0.5, nrm, nrm.clone(), tol=0.0),
        lambda: rp.fredholm_solve(xd, s.tri, s.off, s.adj, nrm, float("nan"), nrm, nrm.clone()),
    ]
    for k, call in enumerate(cases):
        with pytest.raises(G.GGEMError) as e:
            call()
        assert e.value.code == G.ggem.E_ARG, k
    rp.close()
    s.close()
