"""Pins of the oracle's grid machinery (Appendix C, Sec. 3.2.2).

Chebyshev transforms and derivatives are checked against numpy's Chebyshev
polynomial routines; the tau Helmholtz solver and the per-mode Stokes solver
against manufactured polynomial solutions built with those routines; the
spread against the closed-form plane integral of rho_g; the DFT against plane
waves; the interpolation against polynomials it must reproduce exactly.
"""
import math

import numpy as np
import numpy.polynomial.chebyshev as C
import pytest

import oracle as O


def test_cheb_transform_of_Tn():
    Ny = 17
    N = Ny - 1
    yb = np.cos(np.pi * np.arange(Ny) / N)
    Cf = O.cheb_forward_matrix(Ny)
    Ci = O.cheb_inverse_matrix(Ny)
    for n in range(Ny):
        e = np.zeros(Ny)
        e[n] = 1.0
        vals = C.chebval(yb, e)
        assert np.abs(Cf @ vals - e).max() < 1e-14
        assert np.abs(Ci @ e - vals).max() < 1e-14


def test_cheb_diff_matches_chebder(rng):
    for Ny in (9, 33, 65):
        a = rng.standard_normal(Ny)
        D = O.cheb_diff_matrix(Ny)
        ref = np.zeros(Ny)
        d1 = C.chebder(a)
        ref[:d1.size] = d1
        assert np.abs(D @ a - ref).max() < 1e-11 * np.abs(ref).max()


def _cheb_d2(a, H):
    out = np.zeros_like(a)
    d2 = C.chebder(a, 2) / H ** 2
    out[:d2.size] = d2
    return out


@pytest.mark.parametrize("lam", [0.0, 0.5, 40.0, 3e3])
def test_helmholtz_tau_manufactured(lam, rng):
    Ny, H = 33, 1.7
    N = Ny - 1
    D2 = O.cheb_diff_matrix(Ny) @ O.cheb_diff_matrix(Ny)
    # exact solution of degree N-2: the tau residual rows vanish identically
    a = np.zeros(Ny, complex)
    a[:N - 1] = (rng.standard_normal(N - 1) + 1j * rng.standard_normal(N - 1)) * np.exp(-0.1 * np.arange(N - 1))
    r = _cheb_d2(a.real, H) + 1j * _cheb_d2(a.imag, H) - lam * a
    gm = C.chebval(-1.0, a.real) + 1j * C.chebval(-1.0, a.imag)
    gp = C.chebval(1.0, a.real) + 1j * C.chebval(1.0, a.imag)
    sol = O.helmholtz_tau(np.array([lam]), r, np.array([gm]), np.array([gp]), H, D2)[0]
    assert np.abs(sol - a).max() < 1e-12 * np.abs(a).max()


def test_helmholtz_tau_full_degree_rows(rng):
    """Degree-N solution: rows 0..N-2 of the ODE and both wall values hold."""
    Ny, H, lam = 25, 0.8, 7.0
    N = Ny - 1
    D2 = O.cheb_diff_matrix(Ny) @ O.cheb_diff_matrix(Ny)
    r = rng.standard_normal(Ny) + 0j
    sol = O.helmholtz_tau(np.array([lam]), r, np.array([0.3]), np.array([-1.1]), H, D2)[0].real
    res = _cheb_d2(sol, H) - lam * sol - r.real
    assert np.abs(res[:N - 1]).max() < 1e-11 * np.abs(r).max()
    assert abs(C.chebval(-1.0, sol) - 0.3) < 1e-12
    assert abs(C.chebval(1.0, sol) + 1.1) < 1e-12


def _grid_for_modes():
    return O.SlitGrid(6.0, 4.0, 1.3, 4.0, 1.0, 8, 8, 21)


def _cv(a, y):
    return C.chebval(y, a.real) + 1j * C.chebval(y, a.imag)


def _cd(a, H, k=1):
    out = np.zeros_like(a)
    d = (C.chebder(a.real, k) + 1j * C.chebder(a.imag, k)) / H ** k
    out[:d.size] = d
    return out


@pytest.mark.parametrize("mode", [(1, 0), (0, 2), (3, 1), (-2, 3), (1, -3)])
def test_stokes_mode_manufactured(mode, rng):
    """A divergence-free polynomial Stokes solution of one Fourier mode is
    recovered exactly: checks the pressure equation, its sign, the influence
    matrix and the recombination of Eq. cheb_sol."""
    g = _grid_for_modes()
    Ny, H = g.Ny, g.H
    N = Ny - 1
    li, mi = mode[0] % g.Nx, mode[1] % g.Nz
    kx, kz = g.kx[li], g.kz[mi]
    k2 = kx * kx + kz * kz
    deg = N - 3

    def poly():
        a = np.zeros(Ny, complex)
        a[:deg] = (rng.standard_normal(deg) + 1j * rng.standard_normal(deg)) * np.exp(-0.3 * np.arange(deg))
        return a

    v = poly()
    v[deg - 1] = 0.0
    psi = poly()
    phi = _cd(v, H) / k2                      # ik.u_perp + v'/H = 0
    u = 1j * kx * phi + 1j * kz * psi
    w = 1j * kz * phi - 1j * kx * psi
    p = poly()
    # force density from -grad p + lap u + F = 0
    Fx = 1j * kx * p - (_cd(u, H, 2) - k2 * u)
    Fy = _cd(p, H) - (_cd(v, H, 2) - k2 * v)
    Fz = 1j * kz * p - (_cd(w, H, 2) - k2 * w)
    Fh = np.zeros((3, Ny, g.Nx, g.Nz), complex)
    gm = np.zeros((3, g.Nx, g.Nz), complex)
    gp = np.zeros((3, g.Nx, g.Nz), complex)
    for c, (F, s) in enumerate(zip((Fx, Fy, Fz), (u, v, w))):
        Fh[c, :, li, mi] = F
        gm[c, li, mi] = _cv(s, -1.0)
        gp[c, li, mi] = _cv(s, 1.0)
    out = O.solve_modes(g, Fh, gm, gp)
    for got, ref in zip(out, (u, v, w, p)):
        assert np.abs(got[:, li, mi] - ref).max() < 1e-11 * np.abs(ref).max()


def test_stokes_zero_mode_manufactured(rng):
    g = _grid_for_modes()
    Ny, H = g.Ny, g.H
    N = Ny - 1
    u = np.zeros(Ny, complex)
    u[:N - 1] = rng.standard_normal(N - 1)
    w = np.zeros(Ny, complex)
    w[:N - 1] = rng.standard_normal(N - 1)
    v = np.zeros(Ny, complex)
    v[0] = 0.37                                 # uniform wall-normal velocity
    p = np.zeros(Ny, complex)
    p[:N] = rng.standard_normal(N)
    Fx = -_cd(u, H, 2)
    Fz = -_cd(w, H, 2)
    Fy = _cd(p, H)
    Fh = np.zeros((3, Ny, g.Nx, g.Nz), complex)
    gm = np.zeros((3, g.Nx, g.Nz), complex)
    gp = np.zeros((3, g.Nx, g.Nz), complex)
    for c, (F, s) in enumerate(zip((Fx, Fy, Fz), (u, v, w))):
        Fh[c, :, 0, 0] = F
        gm[c, 0, 0] = _cv(s, -1.0)
        gp[c, 0, 0] = _cv(s, 1.0)
    gauge = _cv(p, -1.0)
    out = O.solve_modes(g, Fh, gm, gp, gauge=gauge)
    for got, ref in zip(out, (u, v, w, p)):
        assert np.abs(got[:, 0, 0] - ref).max() < 1e-11 * max(np.abs(ref).max(), 1.0)


def test_nyquist_and_plane_wave():
    g = O.SlitGrid(6.0, 4.0, 1.0, 4.0, 1.0, 16, 12, 9)
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    a = np.cos(2 * np.pi * 3 * X / g.Lx) + 0.5 * np.sin(2 * np.pi * 2 * Z / g.Lz)
    a += 0.25 * np.cos(np.pi * g.Nx * X / g.Lx)   # Nyquist in x
    ah = O.dft_xz(g, a)
    ref = np.zeros_like(ah)
    ref[3, 0] = ref[-3, 0] = 0.5
    ref[0, 2] = -0.25j
    ref[0, -2] = 0.25j
    assert np.abs(ah - ref).max() < 1e-15
    back = O.idft_xz(g, ah)
    assert np.abs(back - (a - 0.25 * np.cos(np.pi * g.Nx * X / g.Lx))).max() < 1e-14


@pytest.mark.parametrize("ys", [0.0, -0.55, 0.31])
def test_spread_plane_integrals(ys):
    """Trapezoid sums of the spread density over each x-z plane equal the
    closed-form plane integral (alpha/sqrt(pi)) (3/2 - alpha^2 s^2)
    exp(-alpha^2 s^2) times the force (r_c = 6/alpha, resolved grid)."""
    alpha = 5.0
    g = O.SlitGrid(3.0, 2.6, 1.0, alpha, 6.0 / alpha, 48, 40, 33)
    xs = np.array([[2.9, ys, 0.05]])                 # straddles both periodic seams
    f = np.array([[0.7, -1.2, 0.4]])
    F = O.spread(g, xs, f)
    sums = F.sum(axis=(2, 3)) * g.dx * g.dz          # (3, Ny)
    s = g.y - ys
    plane = alpha / math.sqrt(math.pi) * (1.5 - alpha ** 2 * s ** 2) * np.exp(-alpha ** 2 * s ** 2)
    inside = np.abs(s) <= 0.6 * g.rc               # planes whose disc is not cut by r_c
    ref = f[0][:, None] * plane[None, :]
    assert np.abs(sums - ref)[:, inside].max() < 1e-9 * np.abs(ref).max()


def test_spread_at_nodes_matches_grid(rng):
    g = O.SlitGrid(4.0, 4.0, 1.0, 3.0, 1.3, 16, 16, 13)
    xs = np.stack([rng.uniform(0, 4, 20), rng.uniform(-0.9, 0.9, 20), rng.uniform(0, 4, 20)], 1)
    f = rng.standard_normal((20, 3))
    F = O.spread(g, xs, f)
    j, i, k = rng.integers(0, 13, 30), rng.integers(0, 16, 30), rng.integers(0, 16, 30)
    got = O.spread_at_nodes(g, xs, f, j, i, k)
    assert np.abs(got - F[:, j, i, k].T).max() < 1e-13 * np.abs(F).max()


def test_interpolation_reproduces_polynomials(rng):
    g = O.SlitGrid(5.0, 4.0, 1.2, 3.0, 1.0, 20, 16, 17)
    X = g.x[None, :, None]
    Y = g.y[:, None, None]
    Z = g.z[None, None, :]

    def poly(x, y, z):
        return 0.3 + x - 0.2 * x ** 2 + 0.05 * x ** 4 + y ** 3 - 0.7 * y ** 4 * z + 0.1 * z ** 4

    field = poly(X, Y, Z)[None]
    # targets away from the periodic seams (the polynomial is not periodic),
    # including the walls and points next to them (clamped y stencil)
    xt = np.stack([rng.uniform(1.0, 3.5, 40), rng.uniform(-1.2, 1.2, 40), rng.uniform(1.0, 2.8, 40)], 1)
    xt[:3, 1] = [-1.2, 1.2, 1.19]
    got = O.interpolate(g, field, xt)[:, 0]
    ref = poly(xt[:, 0], xt[:, 1], xt[:, 2])
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    # a mesh node returns the node value
    node = np.array([[g.x[7], g.y[5], g.z[3]]])
    assert abs(O.interpolate(g, field, node)[0, 0] - field[0, 5, 7, 3]) < 1e-13
