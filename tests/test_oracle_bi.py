"""Pins of the boundary-integral oracle (oracle/bi.py): the element
quadrature of Sec. 3.4.1 (Eq. int_l) and the rigid-particle system of
Sec. 6.1 (Eq. sl_r), each against something other than the oracle itself."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
import oracle.bi as bi
from workloads.inputs import icosphere


def test_regular_rule_exact_for_polynomials():
    """The collapsed 4 x 4 Gauss-Legendre product rule integrates every
    monomial xi^a eta^b of total degree <= 6 over the parent triangle
    exactly: a! b! / (a + b + 2)!."""
    xi, eta, w = bi.triangle_rule(4)
    for a in range(7):
        for b in range(7 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(w * xi ** a * eta ** b) - exact) < 1e-15
    # degree 8 is beyond it
    assert abs(np.sum(w * xi ** 8) - math.factorial(8) / math.factorial(10)) > 1e-10


def test_polar_rule_area():
    """The polar rule about a vertex integrates 1 (area 1/2) only
    approximately at 4 x 4 (the theta integrand 1/(2 (cos + sin)^2) is not a
    polynomial) and converges to it."""
    _, _, w4 = bi.triangle_rule(4, polar=True)
    _, _, w40 = bi.triangle_rule(40, polar=True)
    assert 1e-8 < abs(np.sum(w4) - 0.5) < 2e-3
    assert abs(np.sum(w40) - 0.5) < 1e-13


def inv_r_integral(p1, p2):
    """Closed form of the integral of 1/r over the flat triangle (0, p1, p2):
    in polar coordinates about 0 it is h [atanh(sin u)] between the edge
    ends, h the distance of the line p1 p2 from 0, u the angle from its foot."""
    t = (p2 - p1) / np.linalg.norm(p2 - p1)
    foot = p1 - np.dot(p1, t) * t
    h = np.linalg.norm(foot)
    s1 = np.dot(p1 - foot, t) / np.linalg.norm(p1)
    s2 = np.dot(p2 - foot, t) / np.linalg.norm(p2)
    return h * (math.atanh(s2) - math.atanh(s1))


@pytest.mark.parametrize("tri", [
    ((0.3, 0.05, 0.0), (0.1, 0.25, 0.02)),
    ((0.02, -0.2, 0.1), (0.25, 0.1, -0.05)),
])
def test_vertex_element_singular_integral(tri):
    """Target at a vertex, alpha -> 0 (G^l -> Oseen): for in-plane d,
    trace(int G dS) = 4 int 1/r dS and n . int G dS . n = int 1/r dS, with
    int 1/r dS in closed form.  The polar 4 x 4 rule is within 0.3 % of it,
    and the same rule refined is exact."""
    p1, p2 = (np.array(p) for p in tri)
    e = np.array([np.zeros(3), p1, p2])
    n = np.cross(p1, p2)
    n /= np.linalg.norm(n)
    exact = inv_r_integral(p1, p2)
    for nq, tol in ((4, 3e-3), (48, 1e-11)):
        B = bi.element_blocks(e, 1e-14, vertex=0, n=nq).sum(axis=0)
        assert abs(np.trace(B) - 4 * exact) < tol * 4 * exact
        assert abs(n @ B @ n - exact) < tol * exact
    # z at the second vertex: the relabelled rule gives the same integral
    B1 = bi.element_blocks(e - p1, 1e-14, vertex=1, n=48).sum(axis=0)
    ex1 = inv_r_integral(-p1, p2 - p1)
    assert abs(np.trace(B1) - 4 * ex1) < 1e-10 * ex1


def test_regular_element_against_adaptive_quadrature():
    """A triangle near (not at) the target: the blocks int phi_v G^l_ij dS
    agree with SciPy's adaptive cubature of the same integrand over the
    parent triangle (4 x 4 rule to 1e-4, 16 x 16 to 1e-10)."""
    alpha = 2.0
    e = np.array([[0.25, 0.05, 0.1], [0.45, 0.1, 0.05], [0.3, 0.3, 0.2]])
    omega = np.linalg.norm(np.cross(e[1] - e[0], e[2] - e[0]))

    def ref(v, i, j):
        def f(xi, eta):
            phi = np.array([1 - xi - eta, xi, eta])
            return phi[v] * O.stokeslet_local(-(phi @ e), alpha)[i, j] * omega
        return integrate.dblquad(f, 0, 1, 0, lambda eta: 1 - eta, epsabs=1e-13, epsrel=1e-12)[0]

    B4 = bi.element_blocks(e, alpha, n=4)
    B16 = bi.element_blocks(e, alpha, n=16)
    scale = np.abs(B16).max()
    for v, i, j in ((0, 0, 0), (1, 0, 1), (2, 2, 1), (1, 1, 1)):
        r = ref(v, i, j)
        assert abs(B16[v, i, j] - r) < 1e-10 * scale
        assert abs(B4[v, i, j] - r) < 1e-4 * scale


@pytest.fixture(scope="module")
def sphere():
    V, F = icosphere(1)
    a, H, L, alpha = 0.3, 0.75, 2.0, 8.0
    xc = np.array([L / 2, 0.0, L / 2])
    nodes = V * a + xc
    g = O.SlitGrid(L, L, H, alpha, 4.0 / alpha, 32, 32, 33)
    return g, nodes, F, xc


def test_local_matrix_matches_local_sum(sphere):
    g, nodes, F, _ = sphere
    f = np.random.default_rng(3).standard_normal(nodes.shape)
    Lm = bi.sl_local_matrix(g, nodes, F).reshape(3 * len(nodes), 3 * len(nodes))
    u = bi.sl_local_elements(g, nodes, F, f)
    assert np.abs(Lm @ f.ravel() - u.ravel()).max() < 1e-14 * np.abs(u).max()


@pytest.fixture(scope="module")
def rigid(sphere):
    g, nodes, F, xc = sphere
    return bi.rigid_matrix(g, nodes, F, xc)


def solve(M, rhs_rows):
    sol = np.linalg.solve(M, np.concatenate([rhs_rows.ravel(), np.zeros(6)]))
    n = (len(sol) - 6) // 3
    return sol[:3 * n].reshape(n, 3), sol[3 * n:3 * n + 3], sol[3 * n + 3:]


def test_rigid_matrix_matches_apply(sphere, rigid):
    g, nodes, F, xc = sphere
    x = np.random.default_rng(4).standard_normal(rigid.shape[0])
    n = len(nodes)
    u, Fo, T = bi.rigid_apply(g, nodes, F, xc, x[:3 * n].reshape(n, 3), x[3 * n:3 * n + 3],
                              x[3 * n + 3:])
    y = rigid @ x
    assert np.abs(y - np.concatenate([u.ravel(), Fo, T])).max() < 1e-13 * np.abs(y).max()


def test_rigid_motion_needs_no_traction(sphere, rigid):
    """Undisturbed flow that is itself a rigid motion: the particle moves
    with it and carries no traction."""
    g, nodes, F, xc = sphere
    U0, W0 = np.array([0.3, -0.2, 0.1]), np.array([0.5, 0.1, -0.4])
    f, U, W = solve(rigid, U0 + np.cross(W0, nodes - xc))
    assert np.abs(U - U0).max() < 1e-12 and np.abs(W - W0).max() < 1e-12
    assert np.abs(f).max() < 1e-11


def test_poiseuille_midplane(sphere, rigid):
    """A sphere centred between the walls in pressure-driven flow: by the
    mirror symmetries of mesh, grid and flow it translates along x only and
    does not rotate, slower than the centre-line velocity (Sec. 6.1).  The
    collapsed product rule is not invariant under a relabelling of a
    triangle's vertices, and the mirror image of a triangle is stored with
    its vertices in another order, so the symmetries hold to the quadrature
    error of the rule (about 1e-5 of the local part), not to rounding."""
    g, nodes, F, xc = sphere
    uinf = bi.poiseuille(nodes, 1.0, g.H)
    f, U, W = solve(rigid, uinf)
    assert 0.5 < U[0] < 1.0
    assert np.abs(U[1:]).max() < 1e-6 and np.abs(W).max() < 1e-6
    A = O.node_areas(nodes, F)
    assert np.abs((A[:, None] * f).sum(axis=0)).max() < 1e-12 * np.abs(A[:, None] * f).sum()


def test_torque_of_a_rotational_traction(sphere):
    """Force and torque rows: for f = W0 x (x - x_c) on a sphere of radius a
    the force vanishes and the torque is sum A r x (W0 x r) ~ (2/3) a^2 A W0
    (the surface integral of |r|^2 I - r r is (8 pi a^4 / 3) I)."""
    g, nodes, F, xc = sphere
    W0 = np.array([0.2, -0.5, 0.3])
    r = nodes - xc
    _, Fo, T = bi.rigid_apply(g, nodes, F, xc, np.cross(W0, r), np.zeros(3), np.zeros(3))
    A = O.node_areas(nodes, F)
    a = np.linalg.norm(r, axis=1).mean()
    assert np.abs(Fo).max() < 1e-12
    assert np.abs(T - (2.0 / 3.0) * a * a * A.sum() * W0).max() < 0.02 * np.abs(T).max()


def test_dl_vertex_element_with_ntilde():
    """Double layer on an element that has z as a vertex, alpha -> 0 (T^l ->
    -6 ddd/r^5), with n~ of Eq. ntilde: in polar coordinates about z the
    in-plane d makes d . n_D = 0, so T n~ = 6 u u (u . n_z)(c + s)/(rho |u|^5)
    (u = c e1 + s e2) and the rho-integral of each basis function is
    elementary.  The remaining theta-integral by SciPy's adaptive quadrature
    is the reference: the polar 4 x 4 rule is within 2e-3 of it (the
    theta-integrand is not a polynomial), 48 x 48 within 1e-10."""
    e = np.array([[0.0, 0.0, 0.0], [0.3, 0.05, 0.0], [0.1, 0.25, 0.02]])
    nz = np.array([0.1, -0.2, 1.0])
    nz /= np.linalg.norm(nz)
    omega = np.linalg.norm(np.cross(e[1], e[2]))

    def ref(v, j, i):
        def f(th):
            c, s = math.cos(th), math.sin(th)
            R = 1.0 / (c + s)
            u = c * e[1] + s * e[2]
            phi_int = (R / 2, c * R * R / 2, s * R * R / 2)[v]
            return 6.0 * omega * (c + s) * (u @ nz) * u[j] * u[i] / np.linalg.norm(u) ** 5 * phi_int
        return integrate.quad(f, 0.0, 0.5 * math.pi, epsabs=1e-14, epsrel=1e-13)[0]

    B4 = bi.element_dl_blocks(e, 1e-14, nz, vertex=0, n=4)
    B48 = bi.element_dl_blocks(e, 1e-14, nz, vertex=0, n=48)
    scale = np.abs(B48).max()
    for v, j, i in ((0, 0, 0), (1, 0, 1), (2, 2, 1), (0, 1, 2), (2, 2, 2)):
        r = ref(v, j, i)
        assert abs(B48[v, j, i] - r) < 1e-10 * scale
        assert abs(B4[v, j, i] - r) < 2e-3 * scale


def test_dl_flat_patch_with_matching_normal_vanishes():
    """With n(z) equal to the element normal, n~ is that normal everywhere
    and every in-plane d has d . n = 0: as alpha -> 0 the double layer of the
    element at its own vertex vanishes (the stresslet's remaining term
    carries alpha^3)."""
    e = np.array([[0.0, 0.0, 0.0], [0.3, 0.05, 0.0], [0.1, 0.25, 0.02]])
    n = np.cross(e[1], e[2])
    n /= np.linalg.norm(n)
    B = bi.element_dl_blocks(e, 1e-14, n, vertex=0, n=4)
    assert np.abs(B).max() < 1e-12
    assert np.abs(bi.element_dl_blocks(e, 1e-14, -n, vertex=0, n=4)).max() < 1e-12


def test_dl_regular_element_against_adaptive_quadrature():
    alpha = 2.0
    e = np.array([[0.25, 0.05, 0.1], [0.45, 0.1, 0.05], [0.3, 0.3, 0.2]])
    nz = np.array([0.3, 0.9, -0.2])
    nz /= np.linalg.norm(nz)
    omega = np.linalg.norm(np.cross(e[1] - e[0], e[2] - e[0]))

    def ref(v, j, i):
        def f(xi, eta):
            phi = np.array([1 - xi - eta, xi, eta])
            return phi[v] * (O.stresslet_local(-(phi @ e), alpha)[j, i] @ nz) * omega
        return integrate.dblquad(f, 0, 1, 0, lambda eta: 1 - eta, epsabs=1e-13, epsrel=1e-12)[0]

    B16 = bi.element_dl_blocks(e, alpha, nz, n=16)
    B4 = bi.element_dl_blocks(e, alpha, nz, n=4)
    scale = np.abs(B16).max()
    for v, j, i in ((0, 0, 0), (1, 0, 1), (2, 2, 1)):
        r = ref(v, j, i)
        assert abs(B16[v, j, i] - r) < 1e-10 * scale
        assert abs(B4[v, j, i] - r) < 1e-3 * scale
