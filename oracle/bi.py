"""Boundary-integral discretisation of the single layer on a triangulated
surface and the rigid-particle problem (oracle; test infrastructure only).

Single layer at the mesh nodes (Sec. 3.4, single layer integral), traction
f linear on flat triangles (basis of Sec. 3.3.1: phi1 = 1 - xi - eta,
phi2 = xi, phi3 = eta):

    w(z) = (1/8pi) [ sum_k int_{S_k} f G^l(z - x) dS            (local)
                     + sum_b G^g(z, x_b) f_b A_b ]               (global)

Local part (Sec. 3.4.1, Eq. int_l): every element within r_c of the node z is integrated
over its parent triangle with the product of two 4-point Gauss-Legendre
rules, xi in [0, 1 - eta] for each eta in [0, 1].  When z is a vertex of the
element, the vertex is mapped to (0, 0) and the parent triangle is written in
polar coordinates xi = rho cos(theta), eta = rho sin(theta), theta in
[0, pi/2], rho in [0, 1/(cos + sin)], with the same 4 x 4 product rule in
(rho, theta): the Jacobian rho removes the 1/r singularity of G^l.

Global part (Sec. 3.4.2, global contribution): the nodal trapezoid rule puts
the strength f_b A_b at node b, A_b one third of the areas of the triangles
at b; the GGEM global problem of these point forces (spread, slit solve with
wall data from their local sum, interpolation) gives the velocity at z.

Double layer at the nodes (Sec. 3.5), normal n(z) of the target (the
area-averaged node normal, Sec. 3.5.2):

    v_j(z) = (1/8pi) [ n_k(z) sum_k int_{S_k} q_i T^l_jik(z - x) dS
                       + n_k(z) sigma^g_jk(z) of the point forces q_b A_b ].

On an element that has z as a vertex the normal outside the integral is
replaced inside it by n~(x) = n_D phi_z + n(z) (1 - phi_z) (Eq. dbl_l1,
Eq. ntilde), n_D the element's unit normal and phi_z the basis function of
the vertex z; that element is integrated with the polar rule.

Rigid particle (Sec. 6.1, Eq. sl_r): U + Omega x (x_b - x_c) + w_b = u_inf(x_b)
at every node, with the force- and torque-free conditions
sum_b A_b f_b = 0 and sum_b A_b (x_b - x_c) x f_b = 0.

Readings where the paper is silent or garbled:
  * the upper limit xi(eta) of the parent-triangle integral is 1 - eta;
  * an element is "within r_c" of z when its nearest vertex is (minimum image
    in x and z); such an element is integrated whole;
  * the torque-free condition uses the same nodal weights A_b as the force;
  * the wall data of the global problem is the local sum of the nodal point
    forces (the same point forces that make the global density);
  * n_D is oriented to the side of n(z) (the sign of the cross product of
    the edges depends on the vertex order); the element with z as a vertex
    takes the polar rule, as in the single layer;
  * the undisturbed Poiseuille flow has centre-line velocity U0 between the
    walls at y = -H and y = +H: u_inf = U0 (1 - y^2/H^2) e_x (Appendix B).
"""
from __future__ import annotations

import math

import numpy as np

from .ggem import GLOBAL, INV_8PI, double_layer, single_layer, stokeslet_local, stresslet_local
from .surface import node_areas


def gauss_legendre01(n):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def triangle_rule(n, polar=False):
    """Points (xi, eta) and weights of the n x n product rule on the parent
    triangle xi, eta >= 0, xi + eta <= 1 (weights sum to its area 1/2 for
    the regular rule).  Regular: eta Gauss-Legendre on [0, 1], xi on
    [0, 1 - eta].  Polar about the vertex (0, 0): theta on [0, pi/2], rho on
    [0, 1/(cos + sin)], the weights carrying the Jacobian rho."""
    t, w = gauss_legendre01(n)
    pts, wts = [], []
    if not polar:
        for tj, wj in zip(t, w):
            for ti, wi in zip(t, w):
                pts.append(((1.0 - tj) * ti, tj))
                wts.append(wi * wj * (1.0 - tj))
    else:
        for tk, wk in zip(t, w):
            theta = 0.5 * math.pi * tk
            c, s = math.cos(theta), math.sin(theta)
            rmax = 1.0 / (c + s)
            for ti, wi in zip(t, w):
                rho = rmax * ti
                pts.append((rho * c, rho * s))
                wts.append((0.5 * math.pi * wk) * (rmax * wi) * rho)
    xi, eta = np.array(pts).T
    return xi, eta, np.array(wts)


def element_blocks(e, alpha, vertex=None, n=4):
    """int over one flat triangle of phi_v(x) G^l(z - x) dS for its three
    vertices v (in the given order), without 1/8pi: (3, 3, 3).

    e: (3, 3) vertex positions relative to the target z (consistent images);
    vertex: the local index of the vertex that is z itself, or None."""
    e = np.asarray(e, dtype=np.float64)
    order = [0, 1, 2] if vertex is None else [(vertex + i) % 3 for i in range(3)]
    e = e[order]                     # z is local vertex 0 in the polar case
    if vertex is not None:
        e[0] = 0.0
    omega = np.linalg.norm(np.cross(e[1] - e[0], e[2] - e[0]))
    xi, eta, wts = triangle_rule(n, polar=vertex is not None)
    phi = np.stack([1.0 - xi - eta, xi, eta], axis=1)          # (q, 3)
    G = stokeslet_local(-(phi @ e), alpha)                      # (q, 3, 3)
    B = np.einsum("q,qv,qij->vij", omega * wts, phi, G)
    out = np.empty_like(B)
    out[order] = B                   # back to the given vertex order
    return out


def element_local(e, fe, alpha, vertex=None, n=4):
    """int over one flat triangle of f(x) G^l(z - x) dS with f linear between
    its nodal values fe (3, 3), without 1/8pi."""
    return np.einsum("vij,vj->i", element_blocks(e, alpha, vertex, n), np.asarray(fe))


def element_dl_blocks(e, alpha, nz, vertex=None, n=4):
    """int over one flat triangle of phi_v(x) T^l_jik(z - x) m_k(x) dS for its
    three vertices v: (3, 3 (j), 3 (i)), without 1/8pi.  m = n(z) (nz) when z
    is not a vertex; when it is (local index `vertex`), m = n~(x) of
    Eq. ntilde and the polar rule about z."""
    e = np.asarray(e, dtype=np.float64)
    nz = np.asarray(nz, dtype=np.float64)
    order = [0, 1, 2] if vertex is None else [(vertex + i) % 3 for i in range(3)]
    e = e[order]
    if vertex is not None:
        e[0] = 0.0
    cr = np.cross(e[1] - e[0], e[2] - e[0])
    omega = np.linalg.norm(cr)
    xi, eta, wts = triangle_rule(n, polar=vertex is not None)
    phi = np.stack([1.0 - xi - eta, xi, eta], axis=1)           # (q, 3)
    T = stresslet_local(-(phi @ e), alpha)                       # (q, 3, 3, 3)
    if vertex is None:
        m = np.broadcast_to(nz, (len(wts), 3))
    else:
        nD = cr / omega
        if nD @ nz < 0.0:
            nD = -nD
        m = phi[:, :1] * nD + (1.0 - phi[:, :1]) * nz
    B = np.einsum("q,qv,qjik,qk->vji", omega * wts, phi, T, m)
    out = np.empty_like(B)
    out[order] = B
    return out


def element_images(g, z, xv):
    """Vertex positions relative to z: the first vertex by the minimum image,
    the others by the minimum image of their offset from the first."""
    e0 = g.min_image(xv[0] - z)
    return np.array([e0, e0 + g.min_image(xv[1] - xv[0]), e0 + g.min_image(xv[2] - xv[0])])


def _local_pairs(g, nodes, tri):
    """(target, element, local vertex index of the target or None) for every
    element within r_c of every node (brute force over all elements)."""
    rc2 = g.rc * g.rc
    for zi, z in enumerate(nodes):
        for k in range(tri.shape[0]):
            dv = g.min_image(nodes[tri[k]] - z)
            if np.min(np.sum(dv * dv, axis=1)) > rc2:
                continue
            hit = np.nonzero(tri[k] == zi)[0]
            yield zi, k, (int(hit[0]) if hit.size else None)


def sl_local_matrix(g, nodes, tri, n=4):
    """Local part as a matrix: w_l[z] = sum_b L[z, :, b, :] f[b], with 1/8pi."""
    nodes = np.asarray(nodes, dtype=np.float64)
    tri = np.asarray(tri)
    L = np.zeros((nodes.shape[0], 3, nodes.shape[0], 3))
    for zi, k, vertex in _local_pairs(g, nodes, tri):
        B = element_blocks(element_images(g, nodes[zi], nodes[tri[k]]), g.alpha, vertex, n)
        for v in range(3):
            L[zi, :, tri[k][v], :] += INV_8PI * B[v]
    return L


def sl_local_elements(g, nodes, tri, f, n=4):
    """(1/8pi) sum over the elements within r_c of every node, at every node."""
    nodes = np.asarray(nodes, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    tri = np.asarray(tri)
    out = np.zeros_like(nodes)
    for zi, k, vertex in _local_pairs(g, nodes, tri):
        out[zi] += INV_8PI * element_local(element_images(g, nodes[zi], nodes[tri[k]]),
                                           f[tri[k]], g.alpha, vertex, n)
    return out


def dl_local_elements(g, nodes, tri, normals, q, n=4):
    """(1/8pi) local double layer of Sec. 3.5.2 over the elements within r_c
    of every node, at every node."""
    nodes = np.asarray(nodes, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    normals = np.asarray(normals, dtype=np.float64)
    tri = np.asarray(tri)
    out = np.zeros_like(nodes)
    for zi, k, vertex in _local_pairs(g, nodes, tri):
        B = element_dl_blocks(element_images(g, nodes[zi], nodes[tri[k]]), g.alpha,
                              normals[zi], vertex, n)
        out[zi] += INV_8PI * np.einsum("vji,vi->j", B, q[tri[k]])
    return out


def dl_global_nodal(g, nodes, tri, normals, q):
    """Global double layer of the nodal trapezoid strengths q_b A_b."""
    A = node_areas(nodes, tri)
    return double_layer(g, nodes, A[:, None] * np.asarray(q, dtype=np.float64), nodes,
                        np.asarray(normals, dtype=np.float64), parts=GLOBAL)


def dl_bi(g, nodes, tri, normals, q, n=4):
    """The discretised double layer n_k(z) (1/8pi) int q_i T_jik dS at the nodes."""
    return dl_local_elements(g, nodes, tri, normals, q, n) + dl_global_nodal(g, nodes, tri,
                                                                             normals, q)


def sl_global_nodal(g, nodes, tri, f):
    """Global part with the nodal trapezoid strengths f_b A_b, at the nodes."""
    A = node_areas(nodes, tri)
    return single_layer(g, nodes, A[:, None] * np.asarray(f, dtype=np.float64), nodes,
                        parts=GLOBAL)


def sl_bi(g, nodes, tri, f, n=4):
    """The discretised single layer (1/8pi) int f G dS at the nodes."""
    return sl_local_elements(g, nodes, tri, f, n) + sl_global_nodal(g, nodes, tri, f)


def poiseuille(x, U0, H):
    """Undisturbed pressure-driven flow between the walls y = -H and y = +H."""
    x = np.asarray(x, dtype=np.float64)
    u = np.zeros_like(x)
    u[:, 0] = U0 * (1.0 - (x[:, 1] / H) ** 2)
    return u


def rigid_apply(g, nodes, tri, xc, f, U, Om):
    """Left-hand side of the rigid-particle system: (velocity rows (n, 3),
    force (3,), torque (3,))."""
    nodes = np.asarray(nodes, dtype=np.float64)
    r = nodes - np.asarray(xc, dtype=np.float64)
    A = node_areas(nodes, tri)
    u = np.asarray(U)[None, :] + np.cross(np.asarray(Om)[None, :], r) + sl_bi(g, nodes, tri, f)
    F = (A[:, None] * f).sum(axis=0)
    T = (A[:, None] * np.cross(r, f)).sum(axis=0)
    return u, F, T


def rigid_matrix(g, nodes, tri, xc, n=4):
    """The (3n + 6) x (3n + 6) matrix of the rigid-particle system (unknowns
    ordered f, U, Omega; rows: velocities, force, torque): the local part
    from sl_local_matrix, the global part column by column (one global
    solve per nodal unit force)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    nn = nodes.shape[0]
    m = 3 * nn + 6
    M = np.zeros((m, m))
    M[:3 * nn, :3 * nn] = sl_local_matrix(g, nodes, tri, n).reshape(3 * nn, 3 * nn)
    for j in range(3 * nn):
        f = np.zeros((nn, 3))
        f.flat[j] = 1.0
        M[:3 * nn, j] += sl_global_nodal(g, nodes, tri, f).ravel()
    r = nodes - np.asarray(xc, dtype=np.float64)
    A = node_areas(nodes, tri)
    for b in range(nn):
        for i in range(3):
            M[3 * b + i, 3 * nn + i] = 1.0                       # U
            e = np.zeros(3)
            e[i] = 1.0
            M[3 * b:3 * b + 3, 3 * nn + 3 + i] = np.cross(e, r[b])  # Omega x r
            M[3 * nn + i, 3 * b + i] = A[b]                      # force
            M[3 * nn + 3:, 3 * b + i] = A[b] * np.cross(r[b], e)   # torque
    return M


def rigid_solve(g, nodes, tri, xc, uinf, n=4):
    """Dense solve of the rigid-particle system: (f (n, 3), U, Omega)."""
    nn = np.asarray(nodes).shape[0]
    M = rigid_matrix(g, nodes, tri, xc, n)
    rhs = np.concatenate([np.asarray(uinf, dtype=np.float64).ravel(), np.zeros(6)])
    sol = np.linalg.solve(M, rhs)
    return sol[:3 * nn].reshape(nn, 3), sol[3 * nn:3 * nn + 3], sol[3 * nn + 3:]
