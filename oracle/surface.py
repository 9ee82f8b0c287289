"""FP64 oracle of the surface quantities of a drop suspension in shear.

TEST INFRASTRUCTURE ONLY (see the package header).

* Node normals: the area-averaged normal of the triangles a node belongs to
  (Sec. 3.5.2), i.e. the normalised sum of their area vectors.
* Node areas: one third of the area of every incident triangle (Sec. 4).
* Cotangent Laplace-Beltrami of the position,
      (Lap_s x)_i = 1/(2 A_i) sum_j (cot a_ij + cot b_ij) (x_j - x_i),
  which equals -(1/A_i) d(Area)/dx_i, and the curvature term
  c_i = div_s n = -(Lap_s x)_i . n_i  (c = 2/R on a sphere of radius R).
* Traction jump of a drop membrane with uniform tension 1/Ca, by virtual
  work as in Sec. 4: the membrane energy is Area/Ca, its nodal force is
  F_p = -(1/Ca) d(Area)/dx_p, and dF_p = -F_p/A_p = -(1/Ca) (Lap_s x)_p
  (-> (1/Ca) c n on a smooth surface).
  Undisturbed simple shear u_inf = (g y, 0, 0) has stress g (e_x e_y + e_y e_x)
  (mu = 1), so f_inf = sigma_inf . n = g (n_y, n_x, 0) (App. B).
* Right-hand side of Eq. qa: b = -(1/4pi) (dF/(lambda + 1) + kappa f_inf),
  kappa = (lambda - 1)/(lambda + 1).
* Velocity of Eq. bi_ua at the nodes: u = u_inf + int q_i G_ji dS, with the
  integral taken at the Gauss points of ``gauss_points``; with the 1/8pi of
  ``single_layer`` the integral is 8 pi times that single layer.
"""
from __future__ import annotations

import numpy as np

from .fredholm import gauss_points, interpolate_to_gauss
from .ggem import single_layer


def node_normals(nodes, tri):
    """Area-averaged unit normals (n, 3) of a closed triangulation."""
    acc = np.zeros_like(nodes)
    for t in tri:
        a, b, c = nodes[t[0]], nodes[t[1]], nodes[t[2]]
        av = np.cross(b - a, c - a)          # twice the area vector
        for v in t:
            acc[v] += av
    return acc / np.linalg.norm(acc, axis=1)[:, None]


def node_areas(nodes, tri):
    """One third of the area of every triangle at each of its corners."""
    area = np.zeros(nodes.shape[0])
    for t in tri:
        a, b, c = nodes[t[0]], nodes[t[1]], nodes[t[2]]
        area[list(t)] += np.linalg.norm(np.cross(b - a, c - a)) / 6.0
    return area


def laplace_beltrami_position(nodes, tri):
    """Cotangent Laplace-Beltrami of the position at every node (n, 3)."""
    acc = np.zeros_like(nodes)
    for t in tri:
        for corner in range(3):
            i, j, k = t[corner], t[(corner + 1) % 3], t[(corner + 2) % 3]
            xi, xj, xk = nodes[i], nodes[j], nodes[k]
            # angle at k faces edge (i, j); angle at j faces edge (i, k)
            ak = xi - xk
            bk = xj - xk
            aj = xi - xj
            bj = xk - xj
            cot_k = np.dot(ak, bk) / np.linalg.norm(np.cross(ak, bk))
            cot_j = np.dot(aj, bj) / np.linalg.norm(np.cross(aj, bj))
            acc[i] += cot_k * (xj - xi) + cot_j * (xk - xi)
    return acc / (2.0 * node_areas(nodes, tri))[:, None]


def curvature(nodes, tri, normals=None):
    """c = div_s n = -(Lap_s x) . n at the nodes."""
    n = node_normals(nodes, tri) if normals is None else normals
    return -np.einsum("ij,ij->i", laplace_beltrami_position(nodes, tri), n)


def drop_rhs(normals, lap, lam, inv_ca, shear):
    """b of Eq. qa for drops with tension 1/Ca in simple shear of rate `shear`;
    lap = (Lap_s x) at the nodes."""
    kappa = (lam - 1.0) / (lam + 1.0)
    df = -inv_ca * lap
    finf = shear * np.stack([normals[:, 1], normals[:, 0], np.zeros(len(normals))], axis=1)
    return -(df / (lam + 1.0) + kappa * finf) / (4.0 * np.pi)


def surface_velocity(g, nodes, tri, q, shear):
    """u = u_inf + int q G dS at the nodes (Eq. bi_ua)."""
    pos, w = gauss_points(nodes, tri)
    u = 8.0 * np.pi * single_layer(g, pos, interpolate_to_gauss(q, tri) * w[:, None], nodes)
    u[:, 0] += shear * nodes[:, 1]
    return u
