"""Pins of the oracle's Fredholm operator pieces (CPU).

The three-point interior Gauss rule integrates linear functions exactly over
each flat triangle (sum = area x value at the centroid) and its weights add up
to the surface area; the operator is the identity when kappa = 0 and linear in
its argument.
"""
import numpy as np

import oracle as O
from workloads import case_small_surface, icosphere


def test_gauss_rule_exact_for_linear(rng):
    V, F = icosphere(2)
    X = V * 1.3 + np.array([0.2, -0.1, 0.5])
    pos, w = O.gauss_points(X, F)
    a, b, c = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    assert abs(w.sum() - area.sum()) < 1e-13 * area.sum()
    coef = rng.standard_normal(4)
    lin = lambda p: coef[0] + p @ coef[1:]  # noqa: E731
    cen = (a + b + c) / 3.0
    assert abs((w * lin(pos)).sum() - (area * lin(cen)).sum()) < 1e-12
    # interpolation of nodal values reproduces a linear field at the Gauss points
    q = np.stack([lin(X), 2 * lin(X), -lin(X)], axis=1)
    qg = O.interpolate_to_gauss(q, F)
    assert np.abs(qg[:, 0] - lin(pos)).max() < 1e-13


def test_fredholm_identity_and_linearity(rng):
    c, tri, nrm, b = case_small_surface(5, ncap=1, level=1, N=32, Ny=17)
    g = O.SlitGrid.from_case(c)
    x = rng.standard_normal(b.shape)
    assert np.abs(O.fredholm_apply(g, c.xt, nrm, tri, 0.0, x) - x).max() == 0.0
    y1 = O.fredholm_apply(g, c.xt, nrm, tri, 0.4, x)
    y2 = O.fredholm_apply(g, c.xt, nrm, tri, 0.4, 2.5 * x)
    assert np.abs(y2 - 2.5 * y1).max() < 1e-12 * np.abs(y2).max()
