"""FP64 oracle of the Fredholm operator of the single-layer density (Eq. qa).

TEST INFRASTRUCTURE ONLY (see the package header).  At each element node x_b
  (A q)_j(x_b) = q_j(x_b) + (kappa_b/4pi) n_k(x_b) sum int q_i(x) T_jik(x_b, x) dS(x),
with q linear on flat triangles (Sec. 3.3.1) and the surface integral taken
with the three interior Gauss points of each triangle (barycentric
(2/3, 1/6, 1/6) and permutations, weight area/3).  The integral equals 8 pi
times the double layer of ``oracle.double_layer`` with point forces q(x_g) w_g
at the Gauss points, so (A q) = q + 2 kappa v.
"""
from __future__ import annotations

import numpy as np

from .ggem import double_layer

BARY = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def gauss_points(nodes, tri):
    """(3 ntri, 3) positions and (3 ntri,) weights of the 3-point rule."""
    a, b, c = nodes[tri[:, 0]], nodes[tri[:, 1]], nodes[tri[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    pos = np.einsum("gk,tkd->tgd", BARY, np.stack([a, b, c], axis=1)).reshape(-1, 3)
    w = np.repeat(area / 3.0, 3)
    return pos, w


def interpolate_to_gauss(q, tri):
    """Linear interpolation of nodal values (n, 3) to the Gauss points."""
    qa, qb, qc = q[tri[:, 0]], q[tri[:, 1]], q[tri[:, 2]]
    return np.einsum("gk,tkd->tgd", BARY, np.stack([qa, qb, qc], axis=1)).reshape(-1, 3)


def fredholm_apply(g, nodes, normals, tri, kappa, x):
    """(I + kappa/4pi D) x at the nodes; kappa scalar or (n,)."""
    pos, w = gauss_points(nodes, tri)
    strengths = interpolate_to_gauss(x, tri) * w[:, None]
    v = double_layer(g, pos, strengths, nodes, normals)
    k = np.asarray(kappa, dtype=np.float64)
    k = k[:, None] if k.ndim else k
    return x + 2.0 * k * v
