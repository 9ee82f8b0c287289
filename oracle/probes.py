"""Velocity, pressure and stress at probes; undisturbed-flow stress and
traction; particle stress (oracle; test infrastructure only).

Probes.  For point forces g^nu (Eq. u_g), at any point x of the slit:
    u = u^l + u^g,  p = p^l + p^g,  sigma = sigma^l + sigma^g,
with the local parts summed over pairs within r_c (minimum image):
    u^l = (1/8pi) sum G^l g,  p^l = (1/8pi) sum P^l . g,
    sigma^l_jk = (1/8pi) sum_i T^l_jik g_i   (Eq. local (a)-(c)),
and the global parts from the slit solve of Appendix C (velocity, pressure
and sigma = -p I + grad u + grad u^T in coefficient space) interpolated with
the 4th-order Lagrange stencil of the velocity (Sec. 3.2.2).  A self pair
adds -(4 alpha/sqrt(pi))/(8pi) g to the velocity only (the smoothed pressure
and stress are odd).  The pressure gauge is the double layer's: the lateral
mean of the total pressure at y = -H is zero.

Undisturbed flows (Appendix B), walls at y = -H and y = +H:
    simple shear:  u = (rate y, 0, 0),  sigma = rate e;
    Poiseuille:    u = (U0 (1 - y^2/H^2), 0, 0),  p = -(2 U0/H^2) x,
                   sigma = (2 U0/H^2) x I - (2 U0 y/H^2) e,
e the symmetric tensor with e_xy = e_yx = 1 (the paper's frame y in [0, 2H]
maps to y + H; its 8 U0/H^2 is 2 U0/H^2 in half-gap units).  The traction is
f_inf = sigma . n.

Particle stress (Sec. 7.1): with mu = 1,
    Sigma^p_ij = (1/V) sum_m int_{S_m} [df_i x_j + (lambda - 1)(u_i n_j + u_j n_i)] dS,
the surface integral taken with the nodal weights A_b (one third of the
areas of the triangles at b), as the global part of the single layer does.
"""
from __future__ import annotations

import numpy as np

from .ggem import (
    INV_8PI, SQRT_PI, _apply_y, _pair_blocks, cheb_diff_matrix, cheb_forward_matrix,
    cheb_inverse_matrix, dft_xz, idft_xz, interpolate, pressure_gauge, pressure_local,
    solve_modes, spread, stokeslet_local, stresslet_local, wall_data,
)
from .surface import node_areas

SHEAR = 0
POISEUILLE = 1
# order of the six stress components
SIGMA = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def global_all(g, xs, f):
    """Global u, v, w, p and the six stress components on the grid, each
    (Ny, Nx, Nz), with the double layer's pressure gauge."""
    Cf, Ci, D = cheb_forward_matrix(g.Ny), cheb_inverse_matrix(g.Ny), cheb_diff_matrix(g.Ny)
    Fh = _apply_y(Cf, dft_xz(g, spread(g, xs, f)))
    gm, gp = wall_data(g, xs, f)
    u, v, w, p = solve_modes(g, Fh, dft_xz(g, gm), dft_xz(g, gp), pressure_gauge(g, xs, f))
    ikx = 1j * g.kx[None, :, None]
    ikz = 1j * g.kz[None, None, :]
    dy = lambda a: _apply_y(D, a) / g.H  # noqa: E731
    sig = (-p + 2.0 * ikx * u, -p + 2.0 * dy(v), -p + 2.0 * ikz * w,
           dy(u) + ikx * v, ikz * u + ikx * w, ikz * v + dy(w))
    back = lambda a: idft_xz(g, _apply_y(Ci, a))  # noqa: E731
    return np.stack([back(a) for a in (u, v, w, p)]), np.stack([back(a) for a in sig])


def local_probe(g, xs, f, xt):
    """Local velocity, pressure and stress (six components) at xt."""
    nt = xt.shape[0]
    u = np.zeros((nt, 3))
    p = np.zeros(nt)
    s = np.zeros((nt, 6))
    self_coef = -(4.0 * g.alpha / SQRT_PI) * INV_8PI
    for t0, ti, si, d, s_ti, s_si in _pair_blocks(g, xt, xs):
        if ti.size:
            fs = f[si]
            np.add.at(u, t0 + ti, INV_8PI * np.einsum("pij,pj->pi", stokeslet_local(d, g.alpha), fs))
            np.add.at(p, t0 + ti, INV_8PI * np.einsum("pj,pj->p", pressure_local(d, g.alpha), fs))
            T = np.einsum("pjik,pi->pjk", stresslet_local(d, g.alpha), fs)
            np.add.at(s, t0 + ti, INV_8PI * np.stack([T[:, a, b] for a, b in SIGMA], axis=1))
        if s_ti.size:
            np.add.at(u, t0 + s_ti, self_coef * f[s_si])
    return u, p, s


def probe_fields(g, xs, f, xt):
    """(u (nt, 3), p (nt,), sigma (nt, 6)) at the probes xt."""
    xs = g.wrap(xs)
    xt = g.wrap(xt)
    g.check_sources(xs)
    g.check_targets(xt)
    f = np.asarray(f, dtype=np.float64)
    ul, pl, sl = local_probe(g, xs, f, xt)
    uvwp, sig = global_all(g, xs, f)
    ug = interpolate(g, uvwp, xt)
    sg = interpolate(g, sig, xt)
    return ul + ug[:, :3], pl + ug[:, 3], sl + sg


def undisturbed_stress(kind, rate, H, x):
    """sigma_inf (n, 3, 3) at the points x (Appendix B)."""
    x = np.asarray(x, dtype=np.float64)
    e = np.zeros((3, 3))
    e[0, 1] = e[1, 0] = 1.0
    if kind == SHEAR:
        return np.broadcast_to(rate * e, (x.shape[0], 3, 3)).copy()
    c = 2.0 * rate / (H * H)
    return c * x[:, 0, None, None] * np.eye(3) - c * x[:, 1, None, None] * e


def undisturbed_traction(kind, rate, H, x, n):
    """f_inf = sigma_inf . n at the points x with normals n."""
    return np.einsum("bij,bj->bi", undisturbed_stress(kind, rate, H, x), np.asarray(n))


def particle_stress(nodes, tri, normals, df, u, lam, volume):
    """Sigma^p (3, 3) of Sec. 7.1 with the nodal weights A_b."""
    A = node_areas(nodes, tri)
    x = np.asarray(nodes, dtype=np.float64)
    df, u, n = (np.asarray(a, dtype=np.float64) for a in (df, u, normals))
    S = np.einsum("b,bi,bj->ij", A, df, x)
    S += (lam - 1.0) * (np.einsum("b,bi,bj->ij", A, u, n) + np.einsum("b,bj,bi->ij", A, u, n))
    return S / volume
