"""Physics pins of the whole oracle on tiny, resolved slit problems.

  * the pair enumeration equals a brute-force loop over periodic images;
  * the lateral mean of the velocity is the closed-form k = 0 slit solution
    (f_x/(Lx Lz)) (H + y_<)(H - y_>)/(2H);
  * no-slip at the walls (Sec. 3.2.2: u^g = -u^l there);
  * the local + global sum does not depend on alpha (GGEM split, Sec. 3.2),
    single and double layer, at mesh nodes where no interpolation enters;
  * reciprocity of the mobility (self-adjointness of the Green's function);
  * Gauss law of the stress: the traction flux through a closed sphere is
    minus the enclosed force;
  * the double layer is the Newtonian stress of the single-layer velocity
    (finite differences of single-layer probes).
"""
import math

import numpy as np
import pytest

import oracle as O


def _rand_sources(rng, n, L, H, margin):
    return np.stack([rng.uniform(0, L, n), rng.uniform(-H + margin, H - margin, n),
                     rng.uniform(0, L, n)], 1)


def test_local_sum_matches_image_loop(rng):
    g = O.SlitGrid(3.0, 2.5, 1.0, 3.5, 1.1, 8, 8, 9)
    xs = _rand_sources(rng, 25, 3.0, 1.0, 0.05)
    xs[:, 2] *= 2.5 / 3.0
    f = rng.standard_normal((25, 3))
    xt = np.vstack([xs[:5], _rand_sources(rng, 30, 3.0, 1.0, 0.0) * [1, 1, 2.5 / 3.0]])
    nrm = rng.standard_normal(xt.shape)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    u_ref = np.zeros((xt.shape[0], 3))
    v_ref = np.zeros((xt.shape[0], 3))
    for t in range(xt.shape[0]):
        for s in range(xs.shape[0]):
            for ix in (-1, 0, 1):
                for iz in (-1, 0, 1):
                    d = xt[t] - xs[s] + np.array([ix * g.Lx, 0.0, iz * g.Lz])
                    r2 = float(d @ d)
                    if r2 == 0.0:
                        u_ref[t] += -4 * g.alpha / math.sqrt(math.pi) / (8 * math.pi) * f[s]
                    elif r2 <= g.rc2:
                        u_ref[t] += O.stokeslet_local(d, g.alpha) @ f[s] / (8 * math.pi)
                        T = O.stresslet_local(d, g.alpha)
                        v_ref[t] += np.einsum("jik,i,k->j", T, f[s], nrm[t]) / (8 * math.pi)
    u = O.single_layer(g, xs, f, xt, parts=O.LOCAL)
    v = O.double_layer(g, xs, f, xt, nrm, parts=O.LOCAL)
    assert np.abs(u - u_ref).max() < 1e-13 * np.abs(u_ref).max()
    assert np.abs(v - v_ref).max() < 1e-13 * np.abs(v_ref).max()


def test_zero_mode_closed_form():
    g = O.SlitGrid(4.0, 4.0, 1.0, 6.0, 1.0, 48, 48, 49)
    xs = np.array([[1.3, 0.2, 2.1]])
    f = np.array([[1.0, 0.5, -0.3]])
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    for j in (5, 16, 24, 40):
        pts = np.stack([X.ravel(), np.full(X.size, g.y[j]), Z.ravel()], 1)
        m = O.single_layer(g, xs, f, pts).mean(axis=0)
        ylo, yhi = min(g.y[j], xs[0, 1]), max(g.y[j], xs[0, 1])
        ref = f[0] / (g.Lx * g.Lz) * (g.H + ylo) * (g.H - yhi) / (2 * g.H)
        assert np.abs(m[[0, 2]] - ref[[0, 2]]).max() < 2e-7 * np.abs(ref).max()
        assert abs(m[1]) < 2e-7 * np.abs(ref).max()


def test_no_slip_at_walls(rng):
    # the wall data -u^l of a source at distance d from a wall varies on the
    # scale d, so the grid must resolve it for the zeroed Nyquist row to be small
    g = O.SlitGrid(4.0, 3.0, 1.0, 5.0, 1.0, 64, 48, 33)
    xs = _rand_sources(rng, 6, 3.0, 1.0, 0.45)
    xs[:2, 1] = [-0.5, 0.55]                 # one source near each wall
    f = rng.standard_normal((6, 3))
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    for yw in (-1.0, 1.0):
        pts = np.stack([X.ravel(), np.full(X.size, yw), Z.ravel()], 1)
        ug = O.single_layer(g, xs, f, pts, parts=O.GLOBAL)
        ul = O.single_layer(g, xs, f, pts, parts=O.LOCAL)
        # only the zeroed Nyquist content of the wall data remains
        assert np.abs(ug + ul).max() < 1e-7 * np.abs(ul).max()


@pytest.fixture(scope="module")
def alpha_pair():
    rng = np.random.default_rng(5)
    xs = _rand_sources(rng, 4, 3.2, 1.0, 0.3)
    f = rng.standard_normal((4, 3))
    g0 = O.SlitGrid(3.2, 3.2, 1.0, 4.0, 1.5, 64, 64, 65)
    j, i, k = rng.integers(0, 65, 40), rng.integers(0, 64, 40), rng.integers(0, 64, 40)
    xt = np.stack([g0.x[i], g0.y[j], g0.z[k]], 1)
    # two sources on mesh nodes are also targets: their self pairs enter
    xs[:2] = [[g0.x[9], g0.y[40], g0.z[50]], [g0.x[60], g0.y[28], g0.z[3]]]
    xt = np.vstack([xt, xs[:2]])
    nrm = rng.standard_normal(xt.shape)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    out = {}
    for a in (4.0, 5.0):
        g = O.SlitGrid(3.2, 3.2, 1.0, a, 6.0 / a, 64, 64, 65)
        out[a] = (O.single_layer(g, xs, f, xt), O.double_layer(g, xs, f, xt, nrm))
    return out


def test_alpha_independence_single_layer(alpha_pair):
    a, b = alpha_pair[4.0][0], alpha_pair[5.0][0]
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_alpha_independence_double_layer(alpha_pair):
    a, b = alpha_pair[4.0][1], alpha_pair[5.0][1]
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_reciprocity():
    g = O.SlitGrid(3.2, 3.2, 1.0, 4.0, 1.5, 48, 48, 49)
    a = np.array([[g.x[7], g.y[30], g.z[11]]])
    b = np.array([[g.x[13], g.y[20], g.z[9]]])
    Mab = np.zeros((3, 3))   # velocity at a due to unit forces at b
    Mba = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros((1, 3))
        e[0, j] = 1.0
        Mab[:, j] = O.single_layer(g, b, e, a)[0]
        Mba[:, j] = O.single_layer(g, a, e, b)[0]
    assert np.abs(Mab - Mba.T).max() < 1e-9 * np.abs(Mab).max()


def _sphere_quadrature(c, R, nth=20, nph=40):
    x, w = np.polynomial.legendre.leggauss(nth)
    ph = 2 * np.pi * np.arange(nph) / nph
    CT, PH = np.meshgrid(x, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    n = np.stack([ST * np.cos(PH), CT, ST * np.sin(PH)], -1).reshape(-1, 3)
    wt = (np.repeat(w, nph) * (2 * np.pi / nph)) * R * R
    return c + R * n, n, wt


def test_stress_gauss_law():
    g = O.SlitGrid(3.2, 3.2, 1.0, 4.0, 1.5, 64, 64, 65)
    c = np.array([1.6, 0.1, 1.7])
    pts, n, wt = _sphere_quadrature(c, 0.45)
    force = np.array([[0.8, -0.5, 0.3]])
    inside = O.double_layer(g, c[None, :] + [[0.05, -0.03, 0.02]], force, pts, n)
    flux = (wt[:, None] * inside).sum(axis=0)
    assert np.abs(flux + force[0]).max() < 1e-4
    outside = O.double_layer(g, np.array([[0.4, -0.5, 0.3]]), force, pts, n)
    assert np.abs((wt[:, None] * outside).sum(axis=0)).max() < 1e-4


def test_double_layer_is_stress_of_single_layer(rng):
    """sigma_xy and sigma_xx - sigma_yy from the double layer (normals e_x,
    e_y) equal finite differences of single-layer velocities."""
    g = O.SlitGrid(3.2, 3.2, 1.0, 4.0, 1.5, 64, 64, 65)
    # probe at mesh nodes; steps of one mesh spacing keep every probe on a node
    i, j, k = 20, 30, 40
    p = np.array([g.x[i], g.y[j], g.z[k]])
    # sources at least 0.7 from both probe lines, so the sampled velocity is
    # smooth along them and the spectral derivatives converge
    per = lambda d: d - 3.2 * np.round(d / 3.2)  # noqa: E731
    xs = np.empty((0, 3))
    while len(xs) < 3:
        s = _rand_sources(rng, 1, 3.2, 1.0, 0.3)
        dx, dy, dz = per(s[0, 0] - p[0]), s[0, 1] - p[1], per(s[0, 2] - p[2])
        if np.hypot(dy, dz) >= 0.7 and np.hypot(dx, dz) >= 0.7:
            xs = np.vstack([xs, s])
    f = rng.standard_normal((3, 3))
    ex, ey = np.eye(3)[0], np.eye(3)[1]
    v = O.double_layer(g, xs, f, np.array([p, p]), np.array([ex, ey]))
    sig_xy = v[0, 1]                     # n = e_x: v_y = sigma_yx
    sxx_minus_syy = v[0, 0] - v[1, 1]
    # spectral-accuracy derivatives through SL on the x line and the y line
    xl = np.stack([g.x, np.full(g.Nx, p[1]), np.full(g.Nx, p[2])], 1)
    ux = O.single_layer(g, xs, f, xl)
    kx = np.fft.fftfreq(g.Nx, 1.0 / g.Nx) * 2 * np.pi / g.Lx
    dux = np.real(np.fft.ifft(1j * kx[:, None] * np.fft.fft(ux, axis=0), axis=0))[i]
    yl = np.stack([np.full(g.Ny, p[0]), g.y, np.full(g.Ny, p[2])], 1)
    uy = O.single_layer(g, xs, f, yl)
    coef = O.cheb_forward_matrix(g.Ny) @ uy
    duy = O.cheb_inverse_matrix(g.Ny) @ (O.cheb_diff_matrix(g.Ny) @ coef) / g.H
    ref_xy = duy[j, 0] + dux[1]
    ref_diff = 2 * (dux[0] - duy[j, 1])
    scale = np.abs(v).max()
    assert abs(sig_xy - ref_xy) < 1e-6 * scale
    assert abs(sxx_minus_syy - ref_diff) < 1e-6 * scale
