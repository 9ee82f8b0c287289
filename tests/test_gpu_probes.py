"""Velocity, pressure and stress at probes, undisturbed-flow traction and
particle stress through the C-ABI, against oracle/probes.py."""
import numpy as np
import pytest

import oracle as O
import oracle.probes as P
from workloads.inputs import icosphere

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402
from paper_1109_6587_amd.drops import incidence  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(31)
    L, H, N, Ny, alpha = 3.2, 1.2, 48, 65, 4.0
    g = O.SlitGrid(L, L, H, alpha, 6.0 / alpha, N, N, Ny)
    ns = 40
    xs = np.stack([rng.uniform(0, L, ns), rng.uniform(-1.1, 1.1, ns), rng.uniform(0, L, ns)], 1)
    f = rng.standard_normal((ns, 3))
    xt = np.stack([rng.uniform(0, L, 30), rng.uniform(-H, H, 30), rng.uniform(0, L, 30)], 1)
    xt[:3] = xs[:3]                                   # coincident with sources
    xt[3, 1], xt[4, 1] = H, -H                        # on the walls
    xt[5] += [-L, 0.0, 2 * L]                         # other periodic images
    xt[6] += [L, 0.0, -L]
    ref = P.probe_fields(g, xs, f, xt)
    return g, xs, f, xt, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_probe_parity(case, precision, tol):
    g, xs, f, xt, (ur, pr, sr) = case
    print(f"probes {precision}", flush=True)
    plan = G.Plan(g.Lx, g.Lz, g.H, g.alpha, g.Nx, g.Nz, g.Ny, rc=g.rc, precision=precision,
                  max_src=len(xs), max_tgt=len(xt))
    u, p, s = (a.cpu().numpy() for a in plan.probe(dev(xs), dev(f), dev(xt)))
    assert np.abs(u - ur).max() < tol * np.abs(ur).max()
    assert np.abs(p - pr).max() < tol * np.abs(pr).max()
    assert np.abs(s - sr).max() < tol * np.abs(sr).max()
    if precision == "fp64":
        # the velocity equals the single layer's at the same points
        ul = plan.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
        assert np.abs(u - ul).max() < 1e-12 * np.abs(ul).max()
    plan.close()


def test_probe_domain_errors(case):
    g, xs, f, xt, _ = case
    plan = G.Plan(g.Lx, g.Lz, g.H, g.alpha, g.Nx, g.Nz, g.Ny, rc=g.rc, precision="fp64",
                  max_src=len(xs), max_tgt=len(xt))
    for bad in ((0.5, 1.3, 0.5), (np.nan, 0.0, 0.5)):
        x = xt.copy()
        x[7] = bad
        with pytest.raises(G.GGEMError) as e:
            plan.probe(dev(xs), dev(f), dev(x))
        assert e.value.code == G.ggem.E_DOMAIN
    with pytest.raises(G.GGEMError):
        G.Plan(g.Lx, g.Lz, g.H, g.alpha, g.Nx, g.Nz, g.Ny, rc=g.rc, max_src=5,
               max_tgt=5).probe(dev(xs), dev(f), dev(xt))
    # more probes than the target capacity: rejected before any device work
    small = G.Plan(g.Lx, g.Lz, g.H, g.alpha, g.Nx, g.Nz, g.Ny, rc=g.rc, max_src=len(xs),
                   max_tgt=len(xt) - 1)
    with pytest.raises(G.GGEMError) as e:
        small.probe(dev(xs), dev(f), dev(xt))
    assert e.value.code == G.ggem.E_CAPACITY and "max_tgt" in str(e.value)
    small.close()
    plan.close()


@pytest.mark.parametrize("kind,rate", [(G.FLOW_SHEAR, 1.3), (G.FLOW_POISEUILLE, 0.7)])
def test_undisturbed_traction(kind, rate):
    plan = G.Plan(4.0, 4.0, 0.8, 4.0, 32, 32, 33, rc=1.0)
    rng = np.random.default_rng(4)
    x = np.stack([rng.uniform(-2, 6, 50), rng.uniform(-0.8, 0.8, 50), rng.uniform(0, 4, 50)], 1)
    n = rng.standard_normal((50, 3))
    out = G.undisturbed_traction(plan, kind, rate, dev(x), dev(n)).cpu().numpy()
    ref = P.undisturbed_traction(kind, rate, 0.8, x, n)
    assert np.abs(out - ref).max() < 1e-14 * np.abs(ref).max()
    plan.close()


def test_particle_stress():
    V, F = icosphere(2)
    x = V * 0.4 + np.array([1.0, 0.1, 1.2])
    off, adj = incidence(F, len(x))
    rng = np.random.default_rng(5)
    nrm = O.node_normals(x, F)
    df, u = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    plan = G.Plan(2.0, 2.0, 0.75, 8.0, 32, 32, 33, rc=0.5, max_src=len(x), max_tgt=len(x))
    rp = G.RigidParticle(plan, len(x), len(F))
    S = np.array(rp.particle_stress(dev(x), dev(F, torch.int32), dev(off, torch.int32),
                                    dev(adj, torch.int32), dev(nrm), dev(df), dev(u), 5.0, 3.0))
    ref = P.particle_stress(x, F, nrm, df, u, 5.0, 3.0)
    assert np.abs(S - ref).max() < 1e-13 * np.abs(ref).max()
    rp.close()
    plan.close()
