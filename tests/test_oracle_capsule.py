"""Pins of the capsule oracle (oracle/capsule.py): the neo-Hookean membrane
traction of Sec. 4, volumes and the volume correction of Sec. 5, gaps and the
overlap correction of Sec. 7.1, the time-step rule of Sec. 5."""
import numpy as np
import pytest

import oracle.capsule as C
from oracle.surface import laplace_beltrami_position, node_areas, node_normals
from workloads.inputs import icosphere


def deformed_sphere(level, seed, amp=0.08):
    V, F = icosphere(level)
    rng = np.random.default_rng(seed)
    X = V * 1.05 + amp * rng.standard_normal(V.shape)
    return V, X, F


def test_reference_state_is_free():
    V, F = icosphere(2)
    f, e = C.membrane_forces(V, V.copy(), F, 2.0)
    assert abs(e) < 1e-14 and np.abs(f).max() < 1e-12


def test_forces_are_minus_the_energy_gradient():
    """Virtual work: the reaction forces are -dE/dx, checked by central
    differences of the total energy (which uses only the principal
    stretches, not their derivatives)."""
    V, X, F = deformed_sphere(1, 3)
    f, _ = C.membrane_forces(V, X, F, 1.7)
    h = 1e-6
    rng = np.random.default_rng(0)
    for p in rng.choice(len(X), 6, replace=False):
        for k in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[p, k] += h
            Xm[p, k] -= h
            d = (C.membrane_forces(V, Xp, F, 1.7)[1] - C.membrane_forces(V, Xm, F, 1.7)[1]) / (2 * h)
            assert abs(-d - f[p, k]) < 1e-7 * np.abs(f).max()


def test_rigid_motion_invariance():
    V, X, F = deformed_sphere(1, 4)
    f, e = C.membrane_forces(V, X, F, 1.0)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    R = R @ np.array([[1, 0, 0], [0, np.cos(1.1), -np.sin(1.1)], [0, np.sin(1.1), np.cos(1.1)]])
    f2, e2 = C.membrane_forces(V, X @ R.T + [3.0, -1.0, 2.0], F, 1.0)
    assert abs(e2 - e) < 1e-12 * e
    assert np.abs(f2 - f @ R.T).max() < 1e-12 * np.abs(f).max()
    # every element's forces have zero sum and zero moment
    for t in F[:20]:
        _, fe = C.element(V[t], X[t], 1.0)
        assert np.abs(fe.sum(0)).max() < 1e-12 * np.abs(fe).max()
        assert np.abs(np.cross(X[t], fe).sum(0)).max() < 1e-12 * np.abs(fe).max()


def test_uniaxial_and_equibiaxial_energy():
    """Closed forms of Eq. WNH: an element stretched by (l, 1) in its plane
    stores A0 (G/2)(l^2 + 1 + 1/l^2 - 3); by (l, l), A0 (G/2)(2 l^2 + l^-4 - 3)."""
    x0 = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.3, 0.8, 0]])
    A0 = 0.4
    for l in (0.8, 1.3, 2.0):
        e, _ = C.element(x0, x0 * [l, 1.0, 1.0], 2.5)
        assert abs(e - A0 * 1.25 * (l * l + 1 + 1 / (l * l) - 3)) < 1e-13
        e, _ = C.element(x0, x0 * l, 2.5)
        assert abs(e - A0 * 1.25 * (2 * l * l + l ** -4 - 3)) < 1e-13


def test_uniform_inflation_is_a_uniform_tension():
    """A mesh inflated uniformly by l carries the isotropic tension
    tau = G (1 - l^-6); its traction jump is then exactly that of a membrane
    of uniform tension tau, -tau Lap_s x (the cotangent form), and on the
    sphere it approaches Laplace's 2 tau / R n."""
    V, F = icosphere(3)
    G, l = 2.0, 1.05
    df, _ = C.membrane_traction(V, l * V, F, G)
    tau = G * (1 - l ** -6)
    ref = -tau * laplace_beltrami_position(l * V, F)
    assert np.abs(df - ref).max() < 1e-12 * np.abs(ref).max()
    n = node_normals(l * V, F)
    assert np.abs(np.einsum("ij,ij->i", df, n).mean() - 2 * tau / l) < 1e-2 * 2 * tau / l


def test_volumes():
    V, F = icosphere(3)
    v = C.volumes(np.vstack([V, 2 * V + 5.0]), np.vstack([F, F + len(V)]), 2)
    assert abs(v[1] - 8 * v[0]) < 1e-12 * v[1]
    assert abs(v[0] / (4 * np.pi / 3) - 1) < 1e-2
    # the regular icosahedron inscribed in the unit sphere: edge 4/sqrt(10 + 2 sqrt 5)
    V0, F0 = icosphere(0)
    a = 4 / np.sqrt(10 + 2 * np.sqrt(5))
    assert abs(C.volumes(V0, F0, 1)[0] - 5 / 12 * (3 + np.sqrt(5)) * a ** 3) < 1e-14
    # a unit cube of 12 outward triangles has volume 1 wherever it is
    P = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=float)
    T = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
                  [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]])
    assert abs(C.volumes(P + [7.0, -2.0, 3.0], T, 1)[0] - 1.0) < 1e-13


def test_volume_correction():
    V, F = icosphere(3)
    X = np.vstack([V, V * 1.01 + [3.0, 0, 0]])
    T = np.vstack([F, F + len(V)])
    v0 = C.volumes(np.vstack([V, V + [3.0, 0, 0]]), T, 2)
    out, moved = C.volume_correct(X, T, node_normals(X, T), 2, v0, 1e-4)
    assert list(moved) == [False, True]
    assert np.array_equal(out[: len(V)], X[: len(V)])
    v = C.volumes(out, T, 2)
    # the shift (V0 - V)/A along the normals is exact to first order: a drift
    # of 3 % falls to second order in it
    before = abs(C.volumes(X, T, 2)[1] / v0[1] - 1)
    assert abs(v[1] / v0[1] - 1) < before ** 2


def test_gaps_and_minimum_separation():
    """Two icosahedral spheres on the line of a vertex direction: the gap is
    the centre distance minus both radii (the facing vertices), also across
    the periodic boundary."""
    V, F = icosphere(2)
    v = V[0] / np.linalg.norm(V[0])
    L = 12.0
    for shift in (0.0, L - 2.5 * v[0] - 1.0):
        X = np.vstack([V + [1.0 + shift, 0, 1.0], V + 2.5 * v + [1.0 + shift, 0, 1.0]])
        X[:, 0] = np.mod(X[:, 0], L)
        g = C.gaps(X, 2, L, L)
        assert abs(g[0, 1] - 0.5) < 1e-12
    T = np.vstack([F, F + len(V)])
    assert C.min_separation(X, T, 2, L, L) == min(0.5, C.min_edge(X, T))
    assert C.time_step(0.1, 0.5, 1.0, 2.0) == pytest.approx(0.0125)


def test_overlap_correction():
    V, F = icosphere(1)
    L, H, hm = 10.0, 3.0, 0.05
    X = np.vstack([V + [5.0, 0, 5.0], V + [6.9, 0.2, 5.1], V + [0.5, 0, 9.6],
                   V + [9.5, 0.1, 9.7], V + [2.0, H - 1.01, 2.0]])
    out, sweeps = C.overlap_correct(X, 5, L, L, H, hm)
    assert sweeps >= 1
    g = C.gaps(out, 5, L, L)
    assert g.min() >= hm * (1 - 1e-9)
    Y = out.reshape(5, -1, 3)
    Xr = X.reshape(5, -1, 3)
    # rigid translations only
    for c in range(5):
        d = Y[c] - Xr[c]
        assert np.abs(d - d[0]).max() < 1e-12
    assert Y[4, :, 1].max() <= H - hm + 1e-12
    # a configuration without violations is left alone
    out2, s2 = C.overlap_correct(out, 5, L, L, H, hm)
    assert s2 == 0 and np.array_equal(out2, out)


def test_traction_rhs_reduces_to_the_drop_form():
    """With the uniform-tension traction the capsule right-hand side is the
    drop one of oracle/surface.py."""
    from oracle.surface import drop_rhs
    V, F = icosphere(2)
    n = node_normals(V, F)
    lap = laplace_beltrami_position(V, F)
    b1 = C.traction_rhs(n, -2.0 * lap, 3.0, 0.7)
    b2 = drop_rhs(n, lap, 3.0, 2.0, 0.7)
    assert np.abs(b1 - b2).max() < 1e-15 * np.abs(b2).max()
    assert node_areas(V, F).sum() > 0
