"""Spectrally accurate evaluation of the global solution off the mesh
(oracle; test infrastructure only).

The global velocity (and, for the double layer, stress) of the slit solve is
a Fourier series in x and z times a Chebyshev series in y (Sec. 3.2.2,
Appendix C):

    u(x, y, z) = sum_{l, m} sum_n u_hat[n, l, m] T_n(y/H) exp(i (k_l x + k_m z)),

with the signed wavenumbers of the mesh and the Nyquist row and column zero.
At the mesh nodes this is the grid value; between them it replaces the
4th-order Lagrange stencil, whose error is O(h^5) (Sec. 3.2.2, last
paragraph), by the spectral accuracy of the solve itself.  The oracle sums
the series directly at every target, O(Nx Nz Ny) per target: small grids only.
"""
from __future__ import annotations

import numpy as np

from .ggem import (
    _apply_y, cheb_diff_matrix, cheb_forward_matrix, dft_xz, local_traction, local_velocity,
    pressure_gauge, solve_modes, spread, wall_data,
)


def global_coefficients(g, xs, f, stress=False):
    """Fourier-Chebyshev coefficients (C, Ny, Nx, Nz) of the global velocity,
    or with ``stress`` of the six stress components (xx, yy, zz, xy, xz, yz)."""
    Fh = _apply_y(cheb_forward_matrix(g.Ny), dft_xz(g, spread(g, xs, f)))
    gm, gp = wall_data(g, xs, f)
    gauge = pressure_gauge(g, xs, f) if stress else 0.0
    u, v, w, p = solve_modes(g, Fh, dft_xz(g, gm), dft_xz(g, gp), gauge)
    if not stress:
        return np.stack([u, v, w])
    D = cheb_diff_matrix(g.Ny)
    ikx = 1j * g.kx[None, :, None]
    ikz = 1j * g.kz[None, None, :]
    dy = lambda a: _apply_y(D, a) / g.H  # noqa: E731
    return np.stack([-p + 2.0 * ikx * u, -p + 2.0 * dy(v), -p + 2.0 * ikz * w,
                     dy(u) + ikx * v, ikz * u + ikx * w, ikz * v + dy(w)])


def evaluate(g, coef, xt):
    """The series with coefficients coef (C, Ny, Nx, Nz) at targets xt (nt, 3)."""
    xt = np.asarray(xt, dtype=np.float64)
    n = np.arange(g.Ny)
    out = np.zeros((xt.shape[0], coef.shape[0]))
    for t, (x, y, z) in enumerate(xt):
        Tn = np.cos(n * np.arccos(np.clip(y / g.H, -1.0, 1.0)))       # T_n(y/H)
        ex = np.exp(1j * g.kx * x)
        ez = np.exp(1j * g.kz * z)
        out[t] = np.real(np.einsum("cnlm,n,l,m->c", coef, Tn, ex, ez))
    return out


def single_layer_spectral(g, xs, f, xt):
    """The single layer with the global part evaluated by its series."""
    xs, xt = g.wrap(xs), g.wrap(xt)
    g.check_sources(xs)
    g.check_targets(xt)
    f = np.asarray(f, dtype=np.float64)
    return local_velocity(g, xs, f, xt) + evaluate(g, global_coefficients(g, xs, f), xt)


def double_layer_spectral(g, xs, q, xt, nrm):
    """The double layer with the global stress evaluated by its series."""
    xs, xt = g.wrap(xs), g.wrap(xt)
    g.check_sources(xs)
    g.check_targets(xt)
    q = np.asarray(q, dtype=np.float64)
    nrm = np.asarray(nrm, dtype=np.float64)
    s = evaluate(g, global_coefficients(g, xs, q, stress=True), xt)
    sig = np.zeros((xt.shape[0], 3, 3))
    for c, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        sig[:, a, b] = sig[:, b, a] = s[:, c]
    return local_traction(g, xs, q, xt, nrm) + np.einsum("tjk,tk->tj", sig, nrm)
