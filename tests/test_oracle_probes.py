"""Pins of the probe, undisturbed-flow and particle-stress oracle
(oracle/probes.py), each against something other than the oracle itself:
the Newtonian constitutive law and the momentum balance by finite
differences, the trace identity of the stress, the pressure gauge, the
closed forms of Appendix B, and the divergence theorem on a sphere."""
import numpy as np
import pytest

import oracle as O
import oracle.probes as P
from workloads.inputs import icosphere


@pytest.fixture(scope="module")
def field():
    rng = np.random.default_rng(21)
    L, H, N, Ny, alpha = 3.2, 1.2, 48, 65, 4.0
    g = O.SlitGrid(L, L, H, alpha, 6.0 / alpha, N, N, Ny)
    xs = np.stack([rng.uniform(0, L, 5), rng.uniform(-0.8, 0.8, 5), rng.uniform(0, L, 5)], 1)
    f = rng.standard_normal((5, 3))
    # probes at least 0.3 from every source
    xt = []
    while len(xt) < 12:
        x = np.array([rng.uniform(0, L), rng.uniform(-1.0, 1.0), rng.uniform(0, L)])
        if np.min(np.linalg.norm(g.min_image(xs - x), axis=1)) > 0.3:
            xt.append(x)
    return g, xs, f, np.array(xt)


def test_pressure_is_minus_one_third_of_the_stress_trace(field):
    """tr sigma = -3p + 2 div u, and div u vanishes (locally exactly,
    globally to the spectral error)."""
    g, xs, f, xt = field
    _, p, s = P.probe_fields(g, xs, f, xt)
    tr = s[:, 0] + s[:, 1] + s[:, 2]
    assert np.abs(p + tr / 3.0).max() < 1e-6 * np.abs(s).max()
    assert np.abs(p).max() > 1e-3 * np.abs(s).max()


def grad_fd(fun, xt, h=1e-3):
    """Central differences of fun(points) -> (n, C) along x, y, z: (n, C, 3)."""
    cols = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        cols.append((fun(xt + e) - fun(xt - e)) / (2 * h))
    return np.stack(cols, axis=-1)


def test_stress_is_the_newtonian_stress_of_the_probe_velocity(field):
    """sigma = -p I + grad u + grad u^T with grad u from central differences
    of the probe velocity: the global stress is differentiated spectrally
    and then interpolated, the velocity interpolated and then differenced,
    so they agree to the interpolation error of a derivative (<= 1e-3)."""
    g, xs, f, xt = field
    u, p, s = P.probe_fields(g, xs, f, xt)
    du = grad_fd(lambda x: P.probe_fields(g, xs, f, x)[0], xt)     # du_i/dx_k
    for c, (a, b) in enumerate(P.SIGMA):
        ref = -p * (a == b) + du[:, a, b] + du[:, b, a]
        assert np.abs(s[:, c] - ref).max() < 1e-3 * np.abs(s).max()


def test_momentum_balance_away_from_sources(field):
    """d sigma_jk / dx_k = 0 where no force acts, to the error of
    differentiating the 4th-order interpolant (about (alpha dx)^4 = 5e-3 of
    the stress here; it does not fall with the difference step)."""
    g, xs, f, xt = field

    def full(x):
        s = P.probe_fields(g, xs, f, x)[2]
        m = np.zeros((x.shape[0], 3, 3))
        for c, (a, b) in enumerate(P.SIGMA):
            m[:, a, b] = m[:, b, a] = s[:, c]
        return m.reshape(x.shape[0], 9)

    ds = grad_fd(full, xt).reshape(xt.shape[0], 3, 3, 3)
    div = np.einsum("njkk->nj", ds)
    scale = np.abs(P.probe_fields(g, xs, f, xt)[2]).max()
    assert np.abs(div).max() < 1e-2 * scale


def test_pressure_gauge_at_the_lower_wall(field):
    """The lateral mean of the total pressure over the nodes of y = -H is 0."""
    g, xs, f, _ = field
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    xt = np.stack([X.ravel(), np.full(X.size, -g.H), Z.ravel()], 1)
    _, p, _ = P.probe_fields(g, xs, f, xt)
    assert abs(p.mean()) < 1e-8 * np.abs(p).max()


@pytest.mark.parametrize("kind,rate", [(P.SHEAR, 1.3), (P.POISEUILLE, 0.7)])
def test_undisturbed_stress(kind, rate):
    """sigma_inf = -p I + grad u + grad u^T of the closed-form velocity and
    pressure of Appendix B (shear: p = 0), it is divergence-free, and the
    traction is sigma . n."""
    H = 0.8
    rng = np.random.default_rng(2)
    x = np.stack([rng.uniform(-2, 2, 6), rng.uniform(-H, H, 6), rng.uniform(-2, 2, 6)], 1)

    def u(x):
        out = np.zeros_like(x)
        out[:, 0] = rate * x[:, 1] if kind == P.SHEAR else rate * (1 - (x[:, 1] / H) ** 2)
        return out

    p = np.zeros(6) if kind == P.SHEAR else -2.0 * rate / H ** 2 * x[:, 0]
    du = grad_fd(u, x, 1e-4)
    ref = -p[:, None, None] * np.eye(3) + du + du.transpose(0, 2, 1)
    S = P.undisturbed_stress(kind, rate, H, x)
    assert np.abs(S - ref).max() < 1e-8
    dS = grad_fd(lambda y: P.undisturbed_stress(kind, rate, H, y).reshape(len(y), 9), x, 1e-4)
    assert np.abs(np.einsum("njkk->nj", dS.reshape(6, 3, 3, 3))).max() < 1e-8
    n = rng.standard_normal((6, 3))
    assert np.allclose(P.undisturbed_traction(kind, rate, H, x, n), np.einsum("bij,bj->bi", S, n))


def test_particle_stress_on_a_sphere():
    """Divergence theorem on a closed surface of volume V: int n_i x_j dS =
    V delta_ij and int (u_i n_j + u_j n_i) dS = 2 E V for u = E x (E
    symmetric), so df = n gives Sigma = I and (df = 0, lambda = 3) gives
    Sigma = 4 E, to the surface quadrature error."""
    V, F = icosphere(3)
    a = 0.7
    x = V * a + np.array([0.3, -0.1, 0.2])
    vol = 4.0 / 3.0 * np.pi * a ** 3
    nrm = O.node_normals(x, F)
    S = P.particle_stress(x, F, nrm, nrm, np.zeros_like(x), 1.0, vol)
    assert np.abs(S - np.eye(3)).max() < 0.01
    E = np.array([[0.3, 0.1, -0.2], [0.1, -0.5, 0.4], [-0.2, 0.4, 0.2]])
    S = P.particle_stress(x, F, nrm, np.zeros_like(x), x @ E.T, 3.0, vol)
    assert np.abs(S - 4.0 * E).max() < 0.03 * np.abs(4.0 * E).max()
