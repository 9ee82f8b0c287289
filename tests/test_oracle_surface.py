"""Pins of the oracle's surface quantities (CPU).

* The cotangent Laplace-Beltrami times the node area is minus the gradient
  of the total mesh area (central differences), which is what makes the
  virtual-work traction jump of a tension membrane.
* Normals of the icosahedron are its vertex directions; node areas add up to
  the surface area; the curvature term of a sphere is 2/R.
* A uniform normal traction on a closed sphere drives no flow (the Stokeslet
  is divergence-free): u = int q G dS ~ 0 for q parallel to n.
"""
import numpy as np
import pytest

import oracle as O
from workloads import icosphere


def total_area(X, F):
    a, b, c = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()


def test_area_gradient_is_cotangent_laplacian(rng):
    V, F = icosphere(1)
    X = V * [1.2, 1.0, 0.85] + 0.03 * rng.standard_normal(V.shape)
    lap = O.laplace_beltrami_position(X, F)
    A = O.node_areas(X, F)
    h = 1e-6
    grad = np.zeros_like(X)
    for p in range(len(X)):
        for d in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[p, d] += h
            Xm[p, d] -= h
            grad[p, d] = (total_area(Xp, F) - total_area(Xm, F)) / (2 * h)
    assert np.abs(A[:, None] * lap + grad).max() < 1e-8
    # translation invariance: the membrane forces add up to zero
    assert np.abs((A[:, None] * lap).sum(axis=0)).max() < 1e-13


def test_normals_areas_sphere_curvature():
    V, F = icosphere(0)
    assert np.abs(O.node_normals(V, F) - V).max() < 1e-15
    V, F = icosphere(3)
    R = 2.0
    X = R * V
    assert abs(O.node_areas(X, F).sum() - total_area(X, F)) < 1e-12
    c = O.curvature(X, F)
    assert abs(c.mean() * R / 2 - 1) < 5e-3
    assert np.sqrt(((c * R / 2 - 1) ** 2).mean()) < 0.03


def test_shear_rhs_and_free_stream():
    V, F = icosphere(1)
    n = O.node_normals(V, F)
    lap = O.laplace_beltrami_position(V, F)
    # kappa = 0 and no tension: nothing to solve for
    assert np.abs(O.drop_rhs(n, lap, 1.0, 0.0, 1.0)).max() == 0
    # kappa f_inf term: lambda = 3 -> kappa = 1/2, f_inf = (n_y, n_x, 0)
    b = O.drop_rhs(n, lap, 3.0, 0.0, 2.0)
    assert np.allclose(b[:, 0], -0.5 * 2.0 * n[:, 1] / (4 * np.pi), atol=1e-15)
    assert np.allclose(b[:, 1], -0.5 * 2.0 * n[:, 0] / (4 * np.pi), atol=1e-15)
    assert np.abs(b[:, 2]).max() == 0


@pytest.mark.slow
def test_uniform_normal_traction_drives_no_flow():
    V, F = icosphere(2)
    X = 0.7 * V + np.array([2.0, 0.1, 2.0])
    g = O.SlitGrid(4.0, 4.0, 1.2, 4.0, 1.0, 48, 48, 33)
    n = O.node_normals(X, F)
    u_n = O.surface_velocity(g, X, F, n, 0.0)
    # a tangential density of the same size does drive flow
    t = np.cross(n, [0.0, 1.0, 0.0])
    u_t = O.surface_velocity(g, X, F, t, 0.0)
    assert np.abs(u_n).max() < 0.02 * np.abs(u_t).max()
    # the undisturbed shear enters as (g y, 0, 0)
    u0 = O.surface_velocity(g, X, F, np.zeros_like(X), 1.5)
    assert np.allclose(u0, np.stack([1.5 * X[:, 1], 0 * X[:, 1], 0 * X[:, 1]], 1), atol=0)
