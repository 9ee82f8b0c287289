"""Pins of the oracle's closed-form kernels against what the mathematics fixes.

G^l, P^l, T^l (Eq. local) and rho_g (Eq. rho_l_g) are checked against
properties they must have, never against a retyped formula:
  * rho_g has unit mass and zero second moment;
  * (G^l, P^l) is a Stokes flow forced by -rho_g away from the pole and is
    divergence-free (Eq. stokes_l with rho_l = delta - rho_g);
  * T^l is the Newtonian stress of (G^l, P^l) (constitutive law under Eq. u_g);
  * G^l -> Oseen tensor as alpha -> 0, and Oseen - G^l -> (4 alpha/sqrt(pi)) I
    as r -> 0 (the self term of the single layer);
  * the plane-integrated rho_g has the primitive ``plane_primitive``.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

import oracle as O


def oseen(d):
    r = np.linalg.norm(d)
    return np.eye(3) / r + np.outer(d, d) / r ** 3


def fd(fun, x, k, h):
    """4th-order central difference of fun along axis k at x."""
    e = np.zeros(3)
    e[k] = h
    return (-fun(x + 2 * e) + 8 * fun(x + e) - 8 * fun(x - e) + fun(x - 2 * e)) / (12 * h)


@pytest.mark.parametrize("alpha", [0.7, 2.0, 6.0])
def test_rho_g_mass_and_second_moment(alpha):
    # the density is below 1e-60 of its peak beyond r = 12/alpha
    top = 12.0 / alpha
    m0 = integrate.quad(lambda r: 4 * math.pi * r * r * O.rho_g(r * r, alpha), 0, top,
                        epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    m2 = integrate.quad(lambda r: 4 * math.pi * r ** 4 * O.rho_g(r * r, alpha), 0, top,
                        epsabs=1e-12, epsrel=0.0, limit=200)[0]
    assert abs(m0 - 1.0) < 1e-12
    assert abs(m2) * alpha ** 2 < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_local_pair_is_stokes_flow(seed):
    rng = np.random.default_rng(seed)
    alpha = 2.3
    d = rng.standard_normal(3)
    d *= rng.uniform(0.3, 2.5) / alpha / np.linalg.norm(d)
    h = 2e-3 / alpha
    G = lambda x: O.stokeslet_local(x, alpha)  # noqa: E731
    P = lambda x: O.pressure_local(x, alpha)   # noqa: E731
    # momentum: -d_i P_j + lap G_ij = 8 pi rho_g delta_ij  (r > 0)
    lap = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        lap += (-G(d + 2 * e) + 16 * G(d + e) - 30 * G(d) + 16 * G(d - e) - G(d - 2 * e)) / (12 * h * h)
    gradP = np.stack([fd(P, d, i, h) for i in range(3)])        # [i, j] = d_i P_j
    res = -gradP + lap - 8 * math.pi * O.rho_g(d @ d, alpha) * np.eye(3)
    scale = np.abs(lap).max() + np.abs(gradP).max()
    assert np.abs(res).max() < 1e-7 * scale
    # continuity: d_i G_ij = 0
    div = sum(fd(G, d, i, h)[i, :] for i in range(3))
    assert np.abs(div).max() < 1e-6 * np.abs(G(d)).max() / np.linalg.norm(d)


@pytest.mark.parametrize("seed", [3, 4])
def test_stresslet_is_newtonian_stress(seed):
    rng = np.random.default_rng(seed)
    alpha = 1.7
    d = rng.standard_normal(3)
    d *= rng.uniform(0.2, 2.5) / alpha / np.linalg.norm(d)
    h = 1e-3 / alpha
    G = lambda x: O.stokeslet_local(x, alpha)  # noqa: E731
    dG = np.stack([fd(G, d, k, h) for k in range(3)])         # [k, i, j] = d_k G_ij
    P = O.pressure_local(d, alpha)
    T_fd = np.zeros((3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                T_fd[i, j, k] = -P[j] * (i == k) + dG[k, i, j] + dG[i, k, j]
    T = O.stresslet_local(d, alpha)
    assert np.abs(T - T_fd).max() < 1e-8 * np.abs(T).max()
    # full symmetry in (i, j, k)
    for perm in [(1, 0, 2), (0, 2, 1), (2, 1, 0)]:
        assert np.abs(T - T.transpose(perm)).max() < 1e-13 * np.abs(T).max()


def test_local_limits():
    rng = np.random.default_rng(7)
    u = rng.standard_normal(3)
    u /= np.linalg.norm(u)
    # alpha -> 0: the local Stokeslet is the free-space Oseen tensor
    d = 0.8 * u
    assert np.abs(O.stokeslet_local(d, 1e-9) - oseen(d)).max() < 1e-8
    # r -> 0: Oseen - G^l -> (4 alpha/sqrt(pi)) I
    alpha = 3.0
    for r in (1e-4, 1e-5):
        diff = oseen(r * u) - O.stokeslet_local(r * u, alpha)
        assert np.abs(diff - 4 * alpha / math.sqrt(math.pi) * np.eye(3)).max() < 50 * alpha ** 3 * r ** 2 + 1e-9


def test_erfc_against_mpmath():
    from scipy.special import erfc
    for x in (1e-3, 0.3, 1.0, 2.5, 4.0, 5.5):
        ref = float(mpmath.erfc(mpmath.mpf(x)))
        assert abs(erfc(x) - ref) <= 4e-16 * ref


@pytest.mark.parametrize("alpha", [1.0, 3.0])
def test_plane_primitive(alpha):
    def plane_density(s):
        return integrate.quad(lambda rho: 2 * math.pi * rho * O.rho_g(rho * rho + s * s, alpha),
                              0, np.inf, epsabs=1e-14, epsrel=1e-12)[0]
    for s in (-1.3 / alpha, -0.2 / alpha, 0.0, 0.9 / alpha):
        h = 1e-3 / alpha
        deriv = (O.plane_primitive(s + h, alpha) - O.plane_primitive(s - h, alpha)) / (2 * h)
        assert abs(deriv - plane_density(s)) < 1e-6 * alpha
    assert abs(O.plane_primitive(-20 / alpha, alpha)) < 1e-15
    assert abs(O.plane_primitive(20 / alpha, alpha) - 1.0) < 1e-15
    assert abs(O.plane_primitive(0.0, alpha) - 0.5) < 1e-15
