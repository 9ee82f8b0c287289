"""Plain FP64 GGEM evaluation in a planar slit (oracle; test infrastructure only).

Geometry and units.  The box is periodic in x (period Lx) and z (period Lz);
no-slip walls sit at y = -H and y = +H (the paper puts them at y = 0 and
y = 2H; the map is y_paper = y + H).  Viscosity is 1.  Point forces g^nu at
x^nu drive the velocity (Eq. u_g a)

    u_i(x) = (1/8pi) sum_nu G_ij(x, x^nu) g^nu_j,

and the stress (Eq. u_g c); the double layer returns the traction n_k sigma_jk
at targets with normal n (Eq. wdbl and Eq. vsigma).

The evaluation follows the GGEM split of Sec. 3.2:
  * local part: the free-space response to rho_l = delta - rho_g (Eq. local,
    Eq. u_loc), summed over pairs closer than r_c with the minimum-image
    convention in x and z (Sec. 3.2.2);
  * global part: the slit Stokes problem forced by sum g rho_g (Eq. stokes_gg)
    with walls u^g = -u^l, solved spectrally (Fourier in x,z; Chebyshev-tau in
    y; influence matrix of Appendix C), then interpolated to the targets with
    4th-order Lagrange polynomials (Sec. 3.2.2, last paragraph).

Readings where the paper is silent (each mirrored in the design notes):
  * a pair with zero separation is a self pair: the singular local term is
    skipped; the single layer adds -(4 alpha/sqrt(pi))/(8 pi) g, the limit of
    G - G^l, so that the result is the regular part of the slit Green's
    function; the double layer adds nothing (the smoothed stress is odd);
  * pairs are included when |d|^2 <= r_c^2, compared in FP64;
  * the global density is sampled pointwise at the grid nodes (no weights);
  * the 2-D DFT carries the factor 1/(Nx Nz); the Nyquist row and column
    (l = -Nx/2, m = -Nz/2) are zeroed;
  * the tau system keeps rows 0..N-2 of the Helmholtz operator and replaces
    rows N-1, N by the two wall values (Appendix C);
  * the pressure equation reads p'' - k^2 p = div F where F is the force
    density (momentum: -grad p + lap u + F = 0);
  * the k = 0 mode: u, w from the Helmholtz problem with k = 0; v linear
    between its wall values; p from p' = F_y (rows 0..N-1) plus a gauge row;
  * gauge (double layer only): the lateral mean of the total pressure at
    y = -H is zero;
  * no tau correction of the divergence.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

LOCAL = 1
GLOBAL = 2
ALL = 3

SQRT_PI = math.sqrt(math.pi)
INV_8PI = 1.0 / (8.0 * math.pi)


# ---------------------------------------------------------------------------
# problem description
# ---------------------------------------------------------------------------

class SlitGrid:
    """Box, split parameter and Fourier x Fourier x Chebyshev grid.

    Nodes: x_i = i Lx/Nx, z_k = k Lz/Nz (equispaced trapezoidal points) and
    Gauss-Lobatto y_j = H cos(pi j/(Ny-1)), j = 0 at y = +H (Sec. 3.2.2).
    """

    def __init__(self, Lx, Lz, H, alpha, rc, Nx, Nz, Ny):
        rc = 4.0 / alpha if (rc is None or rc == 0) else rc
        if not (H > 0 and alpha > 0 and rc > 0):
            raise ValueError("H, alpha and r_c must be positive")
        if not (rc < 0.5 * min(Lx, Lz)):
            # periodicity of the local sum needs r_c < L/2 (alpha L > 8 at r_c = 4/alpha)
            raise ValueError("r_c must be smaller than half the period")
        if Nx % 2 or Nz % 2 or Nx < 8 or Nz < 8 or Ny < 5:
            raise ValueError("grid: Nx, Nz even and >= 8, Ny >= 5")
        self.Lx, self.Lz, self.H = float(Lx), float(Lz), float(H)
        self.alpha, self.rc = float(alpha), float(rc)
        self.rc2 = self.rc * self.rc
        self.Nx, self.Nz, self.Ny = int(Nx), int(Nz), int(Ny)
        self.N = self.Ny - 1
        self.dx = self.Lx / self.Nx
        self.dz = self.Lz / self.Nz
        self.x = np.arange(self.Nx) * self.dx
        self.z = np.arange(self.Nz) * self.dz
        self.y = self.H * np.cos(np.pi * np.arange(self.Ny) / self.N)
        l = np.fft.fftfreq(self.Nx, 1.0 / self.Nx)
        m = np.fft.fftfreq(self.Nz, 1.0 / self.Nz)
        self.kx = 2.0 * np.pi * l / self.Lx
        self.kz = 2.0 * np.pi * m / self.Lz

    @classmethod
    def from_case(cls, c):
        return cls(c.Lx, c.Lz, c.H, c.alpha, c.rc, c.Nx, c.Nz, c.Ny)

    # -- input handling (boundary contract) --------------------------------
    def wrap(self, x):
        x = np.array(x, dtype=np.float64, copy=True)
        x[:, 0] = np.mod(x[:, 0], self.Lx)
        x[:, 2] = np.mod(x[:, 2], self.Lz)
        x[x[:, 0] >= self.Lx, 0] = 0.0
        x[x[:, 2] >= self.Lz, 2] = 0.0
        return x

    def check_sources(self, xs):
        if not np.all(np.isfinite(xs)):
            raise ValueError("non-finite source position")
        if np.any(np.abs(xs[:, 1]) >= self.H):
            raise ValueError("source outside the slit (|y| >= H)")

    def check_targets(self, xt):
        if not np.all(np.isfinite(xt)):
            raise ValueError("non-finite target position")
        if np.any(np.abs(xt[:, 1]) > self.H):
            raise ValueError("target outside the slit (|y| > H)")

    def min_image(self, d):
        """Minimum-image displacement in the periodic directions (Sec. 3.2.2)."""
        d = np.array(d, dtype=np.float64, copy=True)
        d[..., 0] -= self.Lx * np.rint(d[..., 0] / self.Lx)
        d[..., 2] -= self.Lz * np.rint(d[..., 2] / self.Lz)
        return d


# ---------------------------------------------------------------------------
# closed-form kernels (Eq. rho_l_g, Eq. local)
# ---------------------------------------------------------------------------

def rho_g(r2, alpha):
    """Global (quasi-Gaussian) density of Eq. rho_l_g(a) at squared distance r2."""
    a2r2 = alpha * alpha * r2
    return alpha ** 3 / math.pi ** 1.5 * np.exp(-a2r2) * (2.5 - a2r2)


def stokeslet_local(d, alpha):
    """G^l_ij of Eq. local(a) for displacement(s) d (..., 3); returns (..., 3, 3)."""
    d = np.asarray(d, dtype=np.float64)
    r2 = np.sum(d * d, axis=-1)
    r = np.sqrt(r2)
    ec = erfc(alpha * r)
    ex = np.exp(-alpha * alpha * r2)
    I = np.eye(3)
    dd = d[..., :, None] * d[..., None, :]
    return ((I / r[..., None, None] + dd / (r ** 3)[..., None, None]) * ec[..., None, None]
            - (2.0 * alpha / SQRT_PI) * (I - dd / r2[..., None, None]) * ex[..., None, None])


def pressure_local(d, alpha):
    """P^l_j of Eq. local(b); returns (..., 3)."""
    d = np.asarray(d, dtype=np.float64)
    r2 = np.sum(d * d, axis=-1)
    r = np.sqrt(r2)
    ec = erfc(alpha * r)
    ex = np.exp(-alpha * alpha * r2)
    return (2.0 * d / (r ** 3)[..., None] * ec[..., None]
            + 4.0 * alpha * d / SQRT_PI * ((1.0 / r2 - alpha * alpha) * ex)[..., None])


def stresslet_local(d, alpha):
    """T^l_ijk of Eq. local(c); returns (..., 3, 3, 3)."""
    d = np.asarray(d, dtype=np.float64)
    r2 = np.sum(d * d, axis=-1)
    r = np.sqrt(r2)
    ec = erfc(alpha * r)
    ex = np.exp(-alpha * alpha * r2)
    I = np.eye(3)
    ddd = d[..., :, None, None] * d[..., None, :, None] * d[..., None, None, :]
    dI = (I[None, :, :] * d[..., :, None, None]          # delta_jk x_i
          + I[:, None, :] * d[..., None, :, None]         # delta_ik x_j
          + I[:, :, None] * d[..., None, None, :])        # delta_ij x_k
    e = lambda a: a[..., None, None, None]  # noqa: E731
    return (-6.0 * ddd / e(r ** 5) * e(ec)
            - 12.0 * alpha / SQRT_PI * ddd / e(r2 * r2) * e(ex)
            + 4.0 * alpha ** 3 / SQRT_PI * (dI - 2.0 * ddd / e(r2)) * e(ex))


def plane_primitive(s, alpha):
    """Integral of rho_g over the half space below height s (plane-integrated
    density integrated from -inf to s): 1/2 (1 + erf(alpha s)) +
    alpha s/(2 sqrt(pi)) exp(-alpha^2 s^2)."""
    s = np.asarray(s, dtype=np.float64)
    return 0.5 * (1.0 + erf(alpha * s)) + alpha * s / (2.0 * SQRT_PI) * np.exp(-(alpha * s) ** 2)


# ---------------------------------------------------------------------------
# local part (Eq. u_loc), pairs within r_c under the minimum-image rule
# ---------------------------------------------------------------------------

def _pair_blocks(g, xt, xs, budget=4_000_000):
    """Yield (t0, ti, si, d, self_ti, self_si) over all target/source pairs.

    Every pair is visited (no neighbour structure); pairs with
    0 < |d|^2 <= r_c^2 are returned with their displacement d = x_t - x_s,
    pairs with |d|^2 == 0 are returned as self pairs.
    """
    ns = xs.shape[0]
    ch = max(1, budget // max(ns, 1))
    for t0 in range(0, xt.shape[0], ch):
        d = g.min_image(xt[t0:t0 + ch, None, :] - xs[None, :, :])
        r2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        ti, si = np.nonzero((r2 > 0.0) & (r2 <= g.rc2))
        s_ti, s_si = np.nonzero(r2 == 0.0)
        yield t0, ti, si, d[ti, si], s_ti, s_si


def local_velocity(g, xs, f, xt):
    """u^l at targets: (1/8pi) sum G^l(x_t - x_s) f_s, plus the self rule."""
    u = np.zeros((xt.shape[0], 3))
    self_coef = -(4.0 * g.alpha / SQRT_PI) * INV_8PI
    for t0, ti, si, d, s_ti, s_si in _pair_blocks(g, xt, xs):
        if ti.size:
            G = stokeslet_local(d, g.alpha)
            np.add.at(u, t0 + ti, INV_8PI * np.einsum("pij,pj->pi", G, f[si]))
        if s_ti.size:
            np.add.at(u, t0 + s_ti, self_coef * f[s_si])
    return u


def local_traction(g, xs, q, xt, nrm):
    """Local double layer: n_k(x_t) (1/8pi) sum T^l_jik(x_t - x_s) q_i (Eq. vsigma_l).

    Self pairs contribute nothing (the smoothed stresslet vanishes at r = 0).
    """
    v = np.zeros((xt.shape[0], 3))
    for t0, ti, si, d, _s_ti, _s_si in _pair_blocks(g, xt, xs):
        if ti.size:
            T = stresslet_local(d, g.alpha)
            v_p = np.einsum("pjik,pi,pk->pj", T, q[si], nrm[t0 + ti])
            np.add.at(v, t0 + ti, INV_8PI * v_p)
    return v


def wall_data(g, xs, f):
    """Wall values of the global problem: u^g = -u^l at y = -H and y = +H.

    Returns (g_minus, g_plus), each (3, Nx, Nz), sampled at the wall nodes.
    """
    X, Z = np.meshgrid(g.x, g.z, indexing="ij")
    out = []
    for yw in (-g.H, g.H):
        pts = np.stack([X.ravel(), np.full(X.size, yw), Z.ravel()], axis=1)
        ul = local_velocity(g, xs, f, pts)
        out.append(-ul.T.reshape(3, g.Nx, g.Nz))
    return out[0], out[1]


# ---------------------------------------------------------------------------
# global density on the grid (pointwise assignment within r_c)
# ---------------------------------------------------------------------------

def spread(g, xs, f):
    """F(node) = sum_s f_s rho_g(node - x_s) over |node - x_s|^2 <= r_c^2.

    Returns (3, Ny, Nx, Nz).  Per source only the index window with every
    per-axis offset within r_c is examined; the ball test decides.
    """
    F = np.zeros((3, g.Ny, g.Nx, g.Nz))
    for s in range(xs.shape[0]):
        dx = g.x - xs[s, 0]
        dx -= g.Lx * np.rint(dx / g.Lx)
        dz = g.z - xs[s, 2]
        dz -= g.Lz * np.rint(dz / g.Lz)
        dy = g.y - xs[s, 1]
        ix = np.nonzero(np.abs(dx) <= g.rc)[0]
        iz = np.nonzero(np.abs(dz) <= g.rc)[0]
        jy = np.nonzero(np.abs(dy) <= g.rc)[0]
        if not (ix.size and iz.size and jy.size):
            continue
        DY, DX, DZ = np.meshgrid(dy[jy], dx[ix], dz[iz], indexing="ij")
        r2 = (DX * DX + DY * DY) + DZ * DZ
        w = np.where(r2 <= g.rc2, rho_g(r2, g.alpha), 0.0)
        blk = np.ix_(jy, ix, iz)
        for c in range(3):
            F[c][blk] += f[s, c] * w
    return F


def spread_at_nodes(g, xs, f, j, i, k):
    """F at the listed nodes (arrays j, i, k) by a direct sum over all sources."""
    out = np.zeros((len(j), 3))
    for n, (jj, ii, kk) in enumerate(zip(j, i, k)):
        node = np.array([g.x[ii], g.y[jj], g.z[kk]])
        d = g.min_image(node[None, :] - xs)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        m = r2 <= g.rc2
        out[n] = (f[m] * rho_g(r2[m], g.alpha)[:, None]).sum(axis=0)
    return out


# ---------------------------------------------------------------------------
# transforms (Eq. u_expn, Eq. fourier)
# ---------------------------------------------------------------------------

def dft_xz(g, a):
    """Normalised 2-D DFT over the last two axes (x, z) with Nyquist zeroed."""
    ah = np.fft.fft2(a, axes=(-2, -1)) / (g.Nx * g.Nz)
    ah[..., g.Nx // 2, :] = 0.0
    ah[..., :, g.Nz // 2] = 0.0
    return ah


def idft_xz(g, ah):
    """Inverse of ``dft_xz`` (sum of the Fourier series at the nodes), real part."""
    return np.real(np.fft.ifft2(ah, axes=(-2, -1)) * (g.Nx * g.Nz))


def _cbar(N):
    c = np.ones(N + 1)
    c[0] = c[N] = 2.0
    return c


def cheb_forward_matrix(Ny):
    """Gauss-Lobatto values -> Chebyshev coefficients:
    a_n = 2/(N cbar_n) sum_j u_j cos(pi n j/N)/cbar_j, cbar_0 = cbar_N = 2."""
    N = Ny - 1
    n = np.arange(Ny)
    cb = _cbar(N)
    return 2.0 / (N * cb[:, None] * cb[None, :]) * np.cos(np.pi * np.outer(n, n) / N)


def cheb_inverse_matrix(Ny):
    """Chebyshev coefficients -> values at y_j: u_j = sum_n a_n cos(pi n j/N)."""
    N = Ny - 1
    n = np.arange(Ny)
    return np.cos(np.pi * np.outer(n, n) / N)


def cheb_diff_matrix(Ny):
    """d/d(ybar) on coefficients: (Da)_n = (2/c_n) sum_{p>n, p+n odd} p a_p,
    c_0 = 2, c_n = 1 otherwise."""
    D = np.zeros((Ny, Ny))
    for n in range(Ny):
        cn = 2.0 if n == 0 else 1.0
        for p in range(n + 1, Ny):
            if (p + n) % 2 == 1:
                D[n, p] = 2.0 * p / cn
    return D


def _apply_y(M, a):
    """Apply an (Ny x Ny) operator along the y axis of a (..., Ny, Nx, Nz) array."""
    return np.einsum("nj,...jab->...nab", M, a)


# ---------------------------------------------------------------------------
# Chebyshev-tau Helmholtz problem and the influence-matrix Stokes solve
# ---------------------------------------------------------------------------

def helmholtz_tau(lam, r, gm, gp, H, D2):
    """Tau solution of a'' - lam a = r on [-H, H] with a(-H) = gm, a(+H) = gp.

    ``lam`` (M,), ``r`` (M, N+1) Chebyshev coefficients, ``gm``, ``gp`` (M,)
    (all complex allowed).  The system is rows 0..N-2 of (D2/H^2 - lam I) a = r
    plus the two wall rows sum (-1)^n a_n = gm and sum a_n = gp; it is solved
    densely.  Returns (M, N+1).
    """
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    M = lam.shape[0]
    N1 = D2.shape[0]
    N = N1 - 1
    A = np.broadcast_to(D2 / (H * H), (M, N1, N1)).copy()
    A[:, np.arange(N1), np.arange(N1)] -= lam[:, None]
    A[:, N - 1, :] = (-1.0) ** np.arange(N1)
    A[:, N, :] = 1.0
    rhs = np.array(np.broadcast_to(r, (M, N1)), dtype=np.complex128)
    rhs[:, N - 1] = gm
    rhs[:, N] = gp
    sol = np.linalg.solve(A, np.stack([rhs.real, rhs.imag], axis=-1))
    return sol[..., 0] + 1j * sol[..., 1]


def solve_modes(g, Fh, gmh, gph, gauge=0.0, chunk=1024):
    """Appendix C: per Fourier mode, pressure then u, v, w Helmholtz problems,
    combined with the two homogeneous problems (b), (c) through the 2x2
    influence matrix so that the velocity is divergence-free at both walls.

    ``Fh`` (3, Ny, Nx, Nz): Chebyshev-Fourier coefficients of the force
    density; ``gmh``/``gph`` (3, Nx, Nz): Fourier coefficients of the wall
    velocities at y = -H / y = +H; ``gauge``: value of the k = 0 pressure at
    y = -H.  Returns coefficient arrays (u, v, w, p), each (Ny, Nx, Nz).
    """
    Ny, Nx, Nz, H = g.Ny, g.Nx, g.Nz, g.H
    N = Ny - 1
    D = cheb_diff_matrix(Ny)
    D2 = D @ D
    sgn = (-1.0) ** np.arange(Ny)          # T_n(-1)
    dsg_m = -sgn * np.arange(Ny) ** 2      # T_n'(-1) = (-1)^(n+1) n^2
    dsg_p = np.arange(Ny) ** 2.0           # T_n'(+1) = n^2

    KX, KZ = np.meshgrid(g.kx, g.kz, indexing="ij")
    kx, kz = KX.ravel(), KZ.ravel()
    lam = kx * kx + kz * kz
    Fm = Fh.reshape(3, Ny, -1)
    gm = gmh.reshape(3, -1)
    gp = gph.reshape(3, -1)
    out = np.zeros((4, Ny, Nx * Nz), dtype=np.complex128)

    li = np.arange(Nx * Nz) // Nz
    mi = np.arange(Nx * Nz) % Nz
    nyq = (li == Nx // 2) | (mi == Nz // 2)
    zero = (li == 0) & (mi == 0)
    work = np.nonzero(~nyq & ~zero)[0]

    def div_wall(u, v, w, ikx, ikz):
        # continuity expression ik_x u + v'/H + ik_z w at y = -H and y = +H
        ikx, ikz = ikx[:, 0], ikz[:, 0]
        cm = ikx * (u @ sgn) + (v @ dsg_m) / H + ikz * (w @ sgn)
        cp = ikx * u.sum(axis=1) + (v @ dsg_p) / H + ikz * w.sum(axis=1)
        return cm, cp

    for c0 in range(0, work.size, chunk):
        idx = work[c0:c0 + chunk]
        L = lam[idx]
        ikx = (1j * kx[idx])[:, None]
        ikz = (1j * kz[idx])[:, None]
        fx, fy, fz = (Fm[c][:, idx].T for c in range(3))       # (M, Ny)
        zeros = np.zeros(idx.size)
        ones = np.ones(idx.size)
        # (a): true forcing and wall velocities, homogeneous pressure walls
        divF = ikx * fx + (fy @ D.T) / H + ikz * fz
        pa = helmholtz_tau(L, divF, zeros, zeros, H, D2)
        ua = helmholtz_tau(L, -fx + ikx * pa, gm[0, idx], gp[0, idx], H, D2)
        va = helmholtz_tau(L, -fy + (pa @ D.T) / H, gm[1, idx], gp[1, idx], H, D2)
        wa = helmholtz_tau(L, -fz + ikz * pa, gm[2, idx], gp[2, idx], H, D2)
        # (b), (c): no forcing, no-slip, unit pressure at y = -H resp. y = +H
        sols = []
        for bm, bp in ((ones, zeros), (zeros, ones)):
            pb = helmholtz_tau(L, np.zeros((idx.size, Ny)), bm, bp, H, D2)
            ub = helmholtz_tau(L, ikx * pb, zeros, zeros, H, D2)
            vb = helmholtz_tau(L, (pb @ D.T) / H, zeros, zeros, H, D2)
            wb = helmholtz_tau(L, ikz * pb, zeros, zeros, H, D2)
            sols.append((ub, vb, wb, pb))
        ca_m, ca_p = div_wall(ua, va, wa, ikx, ikz)
        cb_m, cb_p = div_wall(*sols[0][:3], ikx, ikz)
        cc_m, cc_p = div_wall(*sols[1][:3], ikx, ikz)
        det = cb_m * cc_p - cc_m * cb_p
        p1 = (-ca_m * cc_p + cc_m * ca_p) / det
        p2 = (-cb_m * ca_p + ca_m * cb_p) / det
        for q, (fa, fb, fc) in enumerate(zip((ua, va, wa, pa), sols[0], sols[1])):
            out[q][:, idx] = (fa + p1[:, None] * fb + p2[:, None] * fc).T

    # k = 0 (the influence matrix is singular there)
    i0 = 0
    fx0, fy0, fz0 = (Fm[c][:, i0] for c in range(3))
    z1 = np.zeros(1)
    out[0][:, i0] = helmholtz_tau(z1, -fx0, gm[0, i0], gp[0, i0], H, D2)[0]
    out[2][:, i0] = helmholtz_tau(z1, -fz0, gm[2, i0], gp[2, i0], H, D2)[0]
    out[1][:, i0] = helmholtz_tau(z1, np.zeros(Ny), gm[1, i0], gp[1, i0], H, D2)[0]
    # pressure: rows 0..N-1 of (D/H) p = F_y, plus p(-H) = gauge
    A = np.zeros((Ny, Ny))
    A[:N] = D[:N] / H
    A[N] = sgn
    rhs = np.concatenate([fy0[:N], [gauge]]).astype(np.complex128)
    sol = np.linalg.solve(A, np.stack([rhs.real, rhs.imag], axis=-1))
    out[3][:, i0] = sol[:, 0] + 1j * sol[:, 1]
    return tuple(o.reshape(Ny, Nx, Nz) for o in out)


def pressure_gauge(g, xs, f):
    """k = 0 pressure value at y = -H that makes the lateral mean of the total
    pressure vanish there: (1/(Lx Lz)) sum_s f_y,s Phi(-(y_s + H))."""
    return float(np.sum(f[:, 1] * plane_primitive(-(xs[:, 1] + g.H), g.alpha)) / (g.Lx * g.Lz))


def global_fields(g, xs, f, stress=False):
    """Global solution on the grid.

    Returns (3, Ny, Nx, Nz) velocity, or, with ``stress``, the six stress
    components (xx, yy, zz, xy, xz, yz) of sigma = -p I + grad u + grad u^T.
    """
    Cf = cheb_forward_matrix(g.Ny)
    Ci = cheb_inverse_matrix(g.Ny)
    D = cheb_diff_matrix(g.Ny)
    F = spread(g, xs, f)
    Fh = _apply_y(Cf, dft_xz(g, F))
    gm, gp = wall_data(g, xs, f)
    gauge = pressure_gauge(g, xs, f) if stress else 0.0
    u, v, w, p = solve_modes(g, Fh, dft_xz(g, gm), dft_xz(g, gp), gauge)
    if not stress:
        return np.stack([idft_xz(g, _apply_y(Ci, a)) for a in (u, v, w)])
    ikx = 1j * g.kx[None, :, None]
    ikz = 1j * g.kz[None, None, :]
    dy = lambda a: _apply_y(D, a) / g.H  # noqa: E731
    sig = (-p + 2.0 * ikx * u,
           -p + 2.0 * dy(v),
           -p + 2.0 * ikz * w,
           dy(u) + ikx * v,
           ikz * u + ikx * w,
           ikz * v + dy(w))
    return np.stack([idft_xz(g, _apply_y(Ci, a)) for a in sig])


# ---------------------------------------------------------------------------
# interpolation (4th-order Lagrange, 5 nodes per axis)
# ---------------------------------------------------------------------------

def _lagrange(t, nodes):
    """Weights of the Lagrange polynomial through ``nodes`` (..., 5) at t (...)."""
    w = np.ones(nodes.shape)
    for q in range(5):
        for p in range(5):
            if p != q:
                w[..., q] *= (t - nodes[..., p]) / (nodes[..., q] - nodes[..., p])
    return w


def interpolate(g, field, xt):
    """Values of grid fields (C, Ny, Nx, Nz) at targets (nt, 3) -> (nt, C).

    Stencil: x nodes i0-2..i0+2 (periodic) with i0 = floor(x/dx + 1/2), z
    likewise; y nodes j0-2..j0+2 with j0 = clamp(rint(arccos(y/H) N/pi), 2,
    N-2).  Indices come from FP64 positions.
    """
    off = np.arange(-2, 3)
    i0 = np.floor(xt[:, 0] / g.dx + 0.5).astype(np.int64)
    k0 = np.floor(xt[:, 2] / g.dz + 0.5).astype(np.int64)
    xi = xt[:, 0] / g.dx - i0
    zi = xt[:, 2] / g.dz - k0
    wx = _lagrange(xi, np.broadcast_to(off.astype(np.float64), (xt.shape[0], 5)))
    wz = _lagrange(zi, np.broadcast_to(off.astype(np.float64), (xt.shape[0], 5)))
    th = np.arccos(xt[:, 1] / g.H)
    j0 = np.clip(np.rint(th * g.N / np.pi).astype(np.int64), 2, g.Ny - 3)
    jj = j0[:, None] + off[None, :]
    wy = _lagrange(xt[:, 1], g.y[jj])
    ii = np.mod(i0[:, None] + off[None, :], g.Nx)
    kk = np.mod(k0[:, None] + off[None, :], g.Nz)
    vals = field[:, jj[:, :, None, None], ii[:, None, :, None], kk[:, None, None, :]]
    wts = wy[:, :, None, None] * wx[:, None, :, None] * wz[:, None, None, :]
    return np.einsum("qtabc,tabc->tq", vals, wts)


# ---------------------------------------------------------------------------
# the two entry points
# ---------------------------------------------------------------------------

def single_layer(g, xs, f, xt, parts=ALL):
    """u(x_t) = (1/8pi) sum_s G^slit(x_t, x_s) f_s by GGEM (local + global)."""
    xs = g.wrap(xs)
    xt = g.wrap(xt)
    g.check_sources(xs)
    g.check_targets(xt)
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros((xt.shape[0], 3))
    if parts & LOCAL:
        u += local_velocity(g, xs, f, xt)
    if parts & GLOBAL:
        u += interpolate(g, global_fields(g, xs, f), xt)
    return u


def double_layer(g, xs, q, xt, nrm, parts=ALL):
    """v_j(x_t) = n_k(x_t) sigma_jk(x_t), sigma the stress of point forces q."""
    xs = g.wrap(xs)
    xt = g.wrap(xt)
    g.check_sources(xs)
    g.check_targets(xt)
    q = np.asarray(q, dtype=np.float64)
    nrm = np.asarray(nrm, dtype=np.float64)
    v = np.zeros((xt.shape[0], 3))
    if parts & LOCAL:
        v += local_traction(g, xs, q, xt, nrm)
    if parts & GLOBAL:
        s = interpolate(g, global_fields(g, xs, q, stress=True), xt)
        S = np.empty((xt.shape[0], 3, 3))
        S[:, 0, 0], S[:, 1, 1], S[:, 2, 2] = s[:, 0], s[:, 1], s[:, 2]
        S[:, 0, 1] = S[:, 1, 0] = s[:, 3]
        S[:, 0, 2] = S[:, 2, 0] = s[:, 4]
        S[:, 1, 2] = S[:, 2, 1] = s[:, 5]
        v += np.einsum("tjk,tk->tj", S, nrm)
    return v
