"""FP64 oracle of neo-Hookean capsules in shear between the walls.

TEST INFRASTRUCTURE ONLY (see the package header).

* Membrane traction jump (Sec. 4).  Every flat triangle carries the
  neo-Hookean energy A0 W with
      W = (G/2) (lambda1^2 + lambda2^2 + 1/(lambda1^2 lambda2^2) - 3)   (Eq. WNH),
  A0 its reference (stress-free) area and lambda1, lambda2 the principal
  stretches of its uniform in-plane deformation.  As in the finite-element
  approach of Charrier, Shrivastava and Wu, the reference and the deformed
  element are each brought into the xy plane by a rigid motion (first vertex
  at the origin, first edge along +x); the displacements of the vertices
  give the displacement gradient of the linear element, F = I + grad u,
  G = F^T F, whose eigenvalues are lambda1^2 and lambda2^2.  The reaction
  forces are the virtual-work derivatives -A0 dW/du_i, formed here through
  the principal stretches (dlambda_k/dF = F e_k e_k^T / lambda_k with e_k the
  eigenvectors of G) and rotated back into the deformed element's plane in
  space.  The force at a node is the sum over its elements, and the traction
  jump is dF_p = -F_p / A_p (Eq. cntr2) with A_p one third of the current
  area of the node's elements.
* Volume of a closed triangulation: (1/6) sum over triangles of
  x_a . (x_b x x_c) (divergence theorem).
* Volume correction (Sec. 5): a capsule whose volume differs from its
  original volume V0 by more than ``tol`` V0 has every node moved along its
  node normal by (V0 - V)/A, A the capsule's area (the reading of the
  correction the paper cites without defining it).
* Minimum node separation h_s^m (Sec. 5): the shortest mesh edge and the
  smallest node-to-node distance between different capsules (minimum image
  in x and z); the time step is gamma_dot dt = 0.5 Ca h_s^m / a.
* Overlap correction (Sec. 7.1): pairs of capsules whose node-to-node gap
  is below h_min are moved apart rigidly along their line of centres, each
  by half the shortfall; a capsule closer than h_min to a wall is moved away
  from it; sweeps repeat until no pair or wall is violated.
"""
from __future__ import annotations

import numpy as np

from .surface import node_areas


def frame2d(a, b, c):
    """Vertices of a triangle in its own plane, (3, 2): a at the origin, b on
    +x, c above the x axis; and the plane's unit vectors t1, t2 in space."""
    e1, e2 = b - a, c - a
    t1 = e1 / np.linalg.norm(e1)
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n)
    t2 = np.cross(n, t1)
    return np.array([[0.0, 0.0], [e1 @ t1, 0.0], [e2 @ t1, e2 @ t2]]), t1, t2


def neo_hookean_w(l1, l2, G):
    """Strain energy per reference area, Eq. WNH."""
    return 0.5 * G * (l1 * l1 + l2 * l2 + 1.0 / (l1 * l1 * l2 * l2) - 3.0)


def element(x0, x, G):
    """Energy A0 W and reaction forces (3, 3) of one flat element with
    reference vertices x0 (3, 3) and deformed vertices x (3, 3)."""
    P, _, _ = frame2d(*x0)
    Q, t1, t2 = frame2d(*x)
    A0 = 0.5 * ((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
    # gradients of the linear shape functions on the reference element
    grad = np.empty((3, 2))
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        grad[i] = [P[j, 1] - P[k, 1], P[k, 0] - P[j, 0]]
    grad /= 2.0 * A0
    U = Q - P
    F = np.eye(2) + U.T @ grad
    lam2, E = np.linalg.eigh(F.T @ F)
    lam = np.sqrt(lam2)
    energy = A0 * neo_hookean_w(lam[0], lam[1], G)
    # dW/dlambda_k for W of Eq. WNH
    dW = G * (lam - 1.0 / (lam ** 3 * lam[::-1] ** 2))
    dWdF = sum(dW[k] / lam[k] * F @ np.outer(E[:, k], E[:, k]) for k in range(2))
    f2 = -A0 * grad @ dWdF.T                  # row i: -A0 dW/du_i
    return energy, np.outer(f2[:, 0], t1) + np.outer(f2[:, 1], t2)


def membrane_forces(ref_nodes, nodes, tri, G):
    """Reaction force at every node (n, 3) and the total energy."""
    F = np.zeros_like(nodes)
    energy = 0.0
    for t in tri:
        e, f = element(ref_nodes[t], nodes[t], G)
        energy += e
        F[t] += f
    return F, energy


def membrane_traction(ref_nodes, nodes, tri, G):
    """Traction jump dF_p = -F_p / A_p at the nodes (Eq. cntr2), and the
    total membrane energy."""
    F, energy = membrane_forces(ref_nodes, nodes, tri, G)
    return -F / node_areas(nodes, tri)[:, None], energy


def traction_rhs(normals, df, lam, shear):
    """b of Eq. qa for a traction jump df in simple shear of rate `shear`."""
    kappa = (lam - 1.0) / (lam + 1.0)
    finf = shear * np.stack([normals[:, 1], normals[:, 0], np.zeros(len(normals))], axis=1)
    return -(df / (lam + 1.0) + kappa * finf) / (4.0 * np.pi)


def volumes(nodes, tri, ncap):
    """Volume of each capsule; capsules are consecutive, equal groups of
    triangles."""
    a, b, c = nodes[tri[:, 0]], nodes[tri[:, 1]], nodes[tri[:, 2]]
    v = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    return v.reshape(ncap, -1).sum(axis=1)


def volume_correct(nodes, tri, normals, ncap, v0, tol):
    """Nodes after the volume correction, and which capsules it moved."""
    npc = nodes.shape[0] // ncap
    v = volumes(nodes, tri, ncap)
    area = node_areas(nodes, tri)
    out = nodes.copy()
    moved = np.zeros(ncap, dtype=bool)
    for c in range(ncap):
        if abs(v[c] - v0[c]) > tol * abs(v0[c]):
            sl = slice(c * npc, (c + 1) * npc)
            out[sl] += (v0[c] - v[c]) / area[sl].sum() * normals[sl]
            moved[c] = True
    return out, moved


def min_edge(nodes, tri):
    """Shortest edge of the triangulation."""
    best = np.inf
    for t in tri:
        for i in range(3):
            best = min(best, np.linalg.norm(nodes[t[i]] - nodes[t[(i + 1) % 3]]))
    return best


def _min_image(d, Lx, Lz):
    d = d.copy()
    d[..., 0] -= Lx * np.rint(d[..., 0] / Lx)
    d[..., 2] -= Lz * np.rint(d[..., 2] / Lz)
    return d


def gaps(nodes, ncap, Lx, Lz):
    """Node-to-node gap of every capsule pair (ncap, ncap; inf on the
    diagonal), by brute force over all node pairs."""
    npc = nodes.shape[0] // ncap
    X = nodes.reshape(ncap, npc, 3)
    g = np.full((ncap, ncap), np.inf)
    for i in range(ncap):
        for j in range(i + 1, ncap):
            d = _min_image(X[i][:, None, :] - X[j][None, :, :], Lx, Lz)
            g[i, j] = g[j, i] = np.sqrt(np.einsum("abk,abk->ab", d, d).min())
    return g


def min_separation(nodes, tri, ncap, Lx, Lz):
    """h_s^m: the shortest edge or the smallest gap between capsules."""
    g = gaps(nodes, ncap, Lx, Lz) if ncap > 1 else np.full((1, 1), np.inf)
    return min(min_edge(nodes, tri), g.min())


def time_step(h, ca, a, shear):
    """gamma_dot dt = 0.5 Ca h_s^m / a (Sec. 5)."""
    return 0.5 * ca * h / (a * shear)


def overlap_correct(nodes, ncap, Lx, Lz, H, h_min, max_sweeps=100):
    """Nodes after the overlap correction, and the number of sweeps that
    moved something.  Per sweep: every pair with gap < h_min (in increasing
    (i, j) order) adds to each capsule half the shortfall along the line of
    centres (minimum image), away from the other; then each capsule closer
    than h_min to a wall is moved away from it by the shortfall; the moves
    are applied together."""
    npc = nodes.shape[0] // ncap
    X = nodes.reshape(ncap, npc, 3).copy()
    sweeps = 0
    for _ in range(max_sweeps):
        g = gaps(X.reshape(-1, 3), ncap, Lx, Lz) if ncap > 1 else np.full((1, 1), np.inf)
        cen = X.mean(axis=1)
        move = np.zeros((ncap, 3))
        for i in range(ncap):
            for j in range(i + 1, ncap):
                if g[i, j] < h_min:
                    e = _min_image(cen[j] - cen[i], Lx, Lz)
                    e /= np.linalg.norm(e)
                    s = 0.5 * (h_min - g[i, j])
                    move[i] -= s * e
                    move[j] += s * e
        for c in range(ncap):
            top, bot = X[c, :, 1].max(), X[c, :, 1].min()
            if top > H - h_min:
                move[c, 1] -= top - (H - h_min)
            elif bot < -H + h_min:
                move[c, 1] += (-H + h_min) - bot
        if not np.any(move):
            break
        X += move[:, None, :]
        sweeps += 1
    return X.reshape(-1, 3), sweeps
