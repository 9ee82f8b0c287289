"""Seeded input generators for the GGEM slit workloads.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in
the order its docstring lists, so the same seed gives the same arrays on any
machine.  Coordinates follow the library convention: periodic box
``x in [0, Lx)``, ``z in [0, Lz)``, no-slip walls at ``y = -H`` and ``y = +H``.

The capsule workloads mirror the paper's geometry (Section 3.3, surface
discretisation): spheres of radius 1 triangulated by recursive subdivision of
an icosahedron, ``20 * 4**k`` triangles and ``10 * 4**k + 2`` vertices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class SlitCase:
    """One evaluation problem: box, split parameter, grid, sources, targets."""

    name: str
    Lx: float
    Lz: float
    H: float
    alpha: float
    rc: float
    Nx: int
    Nz: int
    Ny: int
    xs: np.ndarray            # (ns, 3) source positions
    f: np.ndarray             # (ns, 3) point-force strengths
    xt: np.ndarray            # (nt, 3) target positions
    normals: np.ndarray | None = None   # (nt, 3) target normals (double layer)
    meta: dict = field(default_factory=dict)

    @property
    def ns(self) -> int:
        return int(self.xs.shape[0])

    @property
    def nt(self) -> int:
        return int(self.xt.shape[0])

    def params(self) -> dict:
        return dict(Lx=self.Lx, Lz=self.Lz, H=self.H, alpha=self.alpha,
                    rc=self.rc, Nx=self.Nx, Nz=self.Nz, Ny=self.Ny)


# ---------------------------------------------------------------------------
# geometry helpers
# ---------------------------------------------------------------------------

def icosphere(level: int):
    """Unit-sphere triangulation by recursive 4-way subdivision of an icosahedron.

    Returns ``(vertices (nv,3), faces (nf,3) int)`` with faces oriented so
    that the cross product of the first two edges points outward.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache: dict = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts)
    F = np.array(faces, dtype=np.int64)
    # orient outward
    e1 = V[F[:, 1]] - V[F[:, 0]]
    e2 = V[F[:, 2]] - V[F[:, 0]]
    cen = V[F].mean(axis=1)
    flip = np.einsum("ij,ij->i", np.cross(e1, e2), cen) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def _place_spheres(rng, n, L, ymax, dmin, max_tries=2_000_000):
    """Random sequential addition of ``n`` centres in the periodic box.

    Draw order per attempt: x, y, z as one ``rng.uniform`` call of shape (3,)
    over ``[0,L) x [-ymax, ymax] x [0,L)``.  A candidate is accepted when its
    minimum-image distance (periodic in x and z only) to every accepted centre
    is at least ``dmin``.
    """
    cen = np.zeros((0, 3))
    tries = 0
    while cen.shape[0] < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("sphere placement did not converge")
        u = rng.uniform(size=3)
        c = np.array([u[0] * L, (2.0 * u[1] - 1.0) * ymax, u[2] * L])
        if cen.shape[0]:
            d = cen - c
            d[:, 0] -= L * np.rint(d[:, 0] / L)
            d[:, 2] -= L * np.rint(d[:, 2] / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < dmin * dmin:
                continue
        cen = np.vstack([cen, c])
    return cen


def _wrap(x, Lx, Lz):
    x = x.copy()
    x[:, 0] = np.mod(x[:, 0], Lx)
    x[:, 2] = np.mod(x[:, 2], Lz)
    # np.mod can return L itself for tiny negative inputs
    x[x[:, 0] >= Lx, 0] = 0.0
    x[x[:, 2] >= Lz, 2] = 0.0
    return x


def smooth_nodes(L, hmax):
    """Smallest even 2^a 3^b 5^c that is >= L / hmax."""
    need = int(math.ceil(L / hmax - 1e-12))
    n = max(need, 8)
    while True:
        if n % 2 == 0:
            m = n
            for p in (2, 3, 5):
                while m % p == 0:
                    m //= p
            if m == 1:
                return n
        n += 1


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def case_small_sl(seed: int = 0) -> SlitCase:
    """64 point forces plus 1,000 probes in a 10 x 2 x 10 slit.

    Draw order: source x,z (one (64,2) uniform draw, scaled by 10); source y
    (uniform on (-0.9, 0.9)); forces (standard normal, (64,3)); probe x,z;
    probe y (uniform on [-1, 1]).  Targets are the sources followed by the
    probes.  alpha = 4, r_c = 1, grid 32 x 32 Fourier x 33 Chebyshev.
    """
    rng = np.random.default_rng(seed)
    L, H = 10.0, 1.0
    ns, npr = 64, 1000
    xz = rng.uniform(size=(ns, 2)) * L
    y = rng.uniform(-0.9, 0.9, size=ns)
    f = rng.standard_normal(size=(ns, 3))
    pxz = rng.uniform(size=(npr, 2)) * L
    py = rng.uniform(-1.0, 1.0, size=npr)
    xs = np.stack([xz[:, 0], y, xz[:, 1]], axis=1)
    xp = np.stack([pxz[:, 0], py, pxz[:, 1]], axis=1)
    xt = np.vstack([xs, xp])
    return SlitCase("small_sl_64", L, L, H, 4.0, 1.0, 32, 32, 33,
                    xs, f, xt, None, dict(seed=seed))


def _capsules(rng, ncap, L, H, level=3):
    V, F = icosphere(level)
    cen = _place_spheres(rng, ncap, L, H - 1.2, 2.2)
    return V, F, cen


def case_capsules_sl(seed: int = 1, ncap: int = 50, L: float = 20.0,
                     H: float = 5.0, Nx: int = 128, Ny: int = 65,
                     alpha: float = 2.0, level: int = 3) -> SlitCase:
    """Single layer on capsule meshes (nodal point forces, force-free capsules).

    Draw order: sphere centres by random sequential addition (see
    ``_place_spheres``; |y_c| <= H - 1.2, centre distance >= 2.2), then nodal
    forces as one standard-normal draw of shape (ncap, nv, 3); the mean over
    each capsule's nodes is removed.  Targets are the sources.
    """
    rng = np.random.default_rng(seed)
    V, F, cen = _capsules(rng, ncap, L, H, level)
    nv = V.shape[0]
    f = rng.standard_normal(size=(ncap, nv, 3))
    f -= f.mean(axis=1, keepdims=True)
    xs = (cen[:, None, :] + V[None, :, :]).reshape(-1, 3)
    xs = _wrap(xs, L, L)
    f = f.reshape(-1, 3)
    return SlitCase(f"capsules_sl_{ncap}x{nv}", L, L, H, alpha, 4.0 / alpha,
                    Nx, Nx, Ny, xs, f, xs.copy(), None,
                    dict(seed=seed, ncap=ncap, nv=nv, centres=cen))


def gauss_points(V, F):
    """Three interior points per triangle at barycentric (2/3,1/6,1/6) and
    permutations; weight = area / 3; normal = the triangle's outward normal."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    bary = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    pts = np.einsum("gk,tkd->tgd", bary, np.stack([a, b, c], axis=1))
    w = np.repeat(area[:, None] / 3.0, 3, axis=1)
    n = np.repeat(nrm[:, None, :], 3, axis=1)
    return pts.reshape(-1, 3), w.reshape(-1), n.reshape(-1, 3)


def case_capsules_dl(seed: int = 2, ncap: int = 400, L: float = 40.0,
                     H: float = 6.0, Nx: int = 256, Ny: int = 65,
                     alpha: float = 2.0, level: int = 3) -> SlitCase:
    """Double layer on capsule meshes: sources and targets are Gauss points.

    Draw order: sphere centres (as in ``case_capsules_sl``), then the density
    q as one normal draw with standard deviation 0.1 of shape
    (ncap * 3 * ntri, 3).  The point-force strength is q times the Gauss
    weight; target normals are the triangles' outward normals.
    """
    rng = np.random.default_rng(seed)
    V, F, cen = _capsules(rng, ncap, L, H, level)
    pts, w, n = gauss_points(V, F)
    ng = pts.shape[0]
    q = rng.normal(0.0, 0.1, size=(ncap * ng, 3))
    xs = (cen[:, None, :] + pts[None, :, :]).reshape(-1, 3)
    xs = _wrap(xs, L, L)
    wts = np.tile(w, ncap)
    nrm = np.tile(n, (ncap, 1))
    g = q * wts[:, None]
    return SlitCase(f"capsules_dl_{ncap}x{ng}", L, L, H, alpha, 4.0 / alpha,
                    Nx, Nx, Ny, xs, g, xs.copy(), nrm,
                    dict(seed=seed, ncap=ncap, ng=ng, centres=cen, q=q, w=wts))


def case_batched(seed: int = 3, n_inst: int = 48, alpha: float = 2.0):
    """Independent slit instances of uneven size.

    Instance i uses ``default_rng([seed, i])`` and draws, in order: the point
    count n_i = round(exp(U(ln 1e3, ln 2e5))), L_i ~ U(8, 40), H_i ~ U(1, 6),
    then sources as in ``case_small_sl`` scaled to (L_i, H_i).  Grid:
    N_x = N_z = smallest even 2^a 3^b 5^c >= L / 0.125 and
    N_y = clamp(ceil(16 H) + 1, 33, 65).  Targets are the sources.
    """
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng([seed, i])
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        L = float(rng.uniform(8.0, 40.0))
        H = float(rng.uniform(1.0, 6.0))
        xz = rng.uniform(size=(n, 2)) * L
        y = rng.uniform(-0.9, 0.9, size=n) * H
        f = rng.standard_normal(size=(n, 3))
        xs = np.stack([xz[:, 0], y, xz[:, 1]], axis=1)
        Nx = smooth_nodes(L, 0.125)
        Ny = int(min(max(math.ceil(16 * H) + 1, 33), 65))
        out.append(SlitCase(f"batched_{i}", L, L, H, alpha, 4.0 / alpha,
                            Nx, Nx, Ny, xs, f, xs.copy(), None,
                            dict(seed=[seed, i])))
    return out


def random_case(seed: int, ns: int, nt: int, L: float, H: float, alpha: float,
                rc: float, Nx: int, Nz: int, Ny: int, Lz: float | None = None,
                ymargin: float = 0.1, dl: bool = False,
                include_sources_as_targets: bool = True) -> SlitCase:
    """Small random problem for tests.

    Draw order: source x, y, z (uniform; |y| <= H - ymargin), strengths
    (standard normal), probe x, y, z (uniform, |y| <= H), then, for the double
    layer, unit normals (normalised standard-normal draws) for all targets.
    """
    Lz = L if Lz is None else Lz
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=(ns, 3))
    xs = np.stack([u[:, 0] * L, (2 * u[:, 1] - 1) * (H - ymargin), u[:, 2] * Lz], axis=1)
    f = rng.standard_normal(size=(ns, 3))
    u = rng.uniform(size=(nt, 3))
    xp = np.stack([u[:, 0] * L, (2 * u[:, 1] - 1) * H, u[:, 2] * Lz], axis=1)
    xt = np.vstack([xs, xp]) if include_sources_as_targets else xp
    nrm = None
    if dl:
        nrm = rng.standard_normal(size=(xt.shape[0], 3))
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return SlitCase(f"random_{seed}", L, Lz, H, alpha, rc, Nx, Nz, Ny,
                    xs, f, xt, nrm, dict(seed=seed))


def node_normals(V, F):
    """Area-averaged node normals of a triangulation (the node normal of the
    paper's double layer, Sec. 3.5.2): sum of the adjacent triangles' area
    vectors, normalised."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    cr = np.cross(b - a, c - a)          # 2 * area * outward normal
    acc = np.zeros_like(V)
    for k in range(3):
        np.add.at(acc, F[:, k], cr)
    return acc / np.linalg.norm(acc, axis=1, keepdims=True)


def case_small_surface(seed: int = 5, ncap: int = 2, level: int = 2, L: float = 8.0,
                       H: float = 2.0, alpha: float = 3.0, N: int = 48, Ny: int = 33):
    """Small triangulated capsule surfaces for Fredholm tests.

    Draw order: sphere centres (as in ``case_capsules_sl``, |y_c| <= H - 1.2,
    centre distance >= 2.2), then a standard-normal right-hand side of shape
    (n_nodes, 3).  Returns (SlitCase with the nodes as targets, triangles,
    node normals, rhs).
    """
    rng = np.random.default_rng(seed)
    V, F = icosphere(level)
    cen = _place_spheres(rng, ncap, L, H - 1.2, 2.2)
    nodes = (cen[:, None, :] + V[None]).reshape(-1, 3)
    tri = (F[None] + (np.arange(ncap) * V.shape[0])[:, None, None]).reshape(-1, 3)
    nrm = node_normals(nodes, tri)
    # positions stay unwrapped so every triangle is contiguous; the evaluation
    # wraps x and z itself
    b = rng.standard_normal(size=nodes.shape)
    c = SlitCase(f"surface_{ncap}x{V.shape[0]}", L, L, H, alpha, 4.0 / alpha, N, N, Ny,
                 nodes, np.zeros_like(nodes), nodes.copy(), nrm, dict(seed=seed))
    return c, tri.astype(np.int32), nrm, b


def _real_sph_harm(l, m, theta, phi):
    """Real spherical harmonic of degree l, order m (theta polar, phi azimuth)."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (np.real(y) if m > 0 else np.imag(y))


@dataclass
class DropCase:
    """Drops in simple shear between walls (the Fredholm workload)."""
    name: str
    Lx: float
    Lz: float
    H: float
    alpha: float
    rc: float
    Nx: int
    Nz: int
    Ny: int
    nodes: np.ndarray        # (ncap * nv, 3) unwrapped positions
    tri: np.ndarray          # (ncap * nf, 3) int32, outward orientation
    ncap: int
    nv: int
    lam: float               # viscosity ratio
    inv_ca: float            # tension / (mu shear a)
    shear: float
    dt: float
    steps: int
    meta: dict


def case_shear_drops(seed: int = 4, level: int = 3, ncap: int = 100, L: float = 16.0,
                     H: float = 4.0, N: int = 64, Ny: int = 33) -> DropCase:
    """100 drops of 642 nodes in a 16 x 8 x 16 slit in simple shear.

    Draw order: the 100 occupied sites of a 6 x 3 x 6 lattice (cell centres in
    x and z, y layers at -2.55, 0, 2.55) as ``rng.choice(108, 100,
    replace=False)``; per site a jitter ``rng.uniform(-1, 1, 3) * (0.1, 0.05,
    0.1)``; per drop the 24 coefficients c_lm ~ N(0, 1) of the real spherical
    harmonics of degrees 1..4 (l-major, m = -l..l), the radial perturbation
    sum c_lm Y_lm scaled so that its largest magnitude over the nodes is 0.1.
    Viscosity ratio 5, Ca = 0.5, shear rate 1, dt = 0.01, 200 steps; alpha = 2.
    """
    rng = np.random.default_rng(seed)
    V, F = icosphere(level)
    sites = np.array([((i + 0.5) * L / 6, y, (k + 0.5) * L / 6)
                      for i in range(6) for y in (-2.55, 0.0, 2.55) for k in range(6)])
    pick = np.sort(rng.choice(len(sites), ncap, replace=False))
    theta = np.arccos(np.clip(V[:, 1], -1, 1))      # polar angle about y
    phi = np.arctan2(V[:, 0], V[:, 2])
    Y = np.stack([_real_sph_harm(l, m, theta, phi) for l in range(1, 5) for m in range(-l, l + 1)],
                 axis=1)
    nodes = []
    for s in pick:
        cen = sites[s] + rng.uniform(-1, 1, 3) * np.array([0.1, 0.05, 0.1])
        pert = Y @ rng.standard_normal(Y.shape[1])
        pert *= 0.1 / np.abs(pert).max()
        nodes.append(cen + V * (1.0 + pert)[:, None])
    nodes = np.concatenate(nodes)
    tri = (F[None] + (np.arange(ncap) * V.shape[0])[:, None, None]).reshape(-1, 3)
    return DropCase(f"shear_drops_{ncap}x{V.shape[0]}", L, L, H, 2.0, 2.0, N, N, Ny, nodes,
                    tri.astype(np.int32), ncap, V.shape[0], 5.0, 2.0, 1.0, 0.01, 200,
                    dict(seed=seed, level=level))


@dataclass
class RigidSphereCase:
    """A rigid sphere between the walls in pressure-driven flow."""

    name: str
    Lx: float
    Lz: float
    H: float
    alpha: float
    rc: float
    Nx: int
    Nz: int
    Ny: int
    nodes: np.ndarray         # (n, 3) mesh nodes
    tri: np.ndarray           # (ntri, 3) int32 triangles (outward)
    center: np.ndarray        # (3,)
    U0: float                 # centre-line velocity of the undisturbed flow
    a: float


def case_rigid_sphere(L: float = 5.0, level: int = 4) -> RigidSphereCase:
    """The rigid-particle validation of Sec. 6.1 (no random draws).

    Walls one unit apart (H = 0.5 here), a sphere of radius a = 0.3
    (confinement 2a over the wall spacing = 0.6) centred between them (the
    paper's y_c/H = 1/2) in Poiseuille flow of centre-line velocity 1;
    level-4 icosphere (5,120 triangles, 2,562 nodes); r_c = 0.5 a = 4/alpha;
    N_y = 61 and equal mean mesh spacings 1/60 in all directions
    (alpha dy_m = 0.44); L_x = L_z = L (the paper takes L = 5 wall spacings
    and extrapolates in L^-2)."""
    H, a = 0.5, 0.3
    rc = 0.5 * a
    N = int(round(L * 60))
    V, F = icosphere(level)
    center = np.array([L / 2, 0.0, L / 2])
    return RigidSphereCase(f"rigid_sphere_L{L:g}", L, L, H, 4.0 / rc, rc, N, N, 61,
                           V * a + center, F.astype(np.int32), center, 1.0, a)


@dataclass
class CapsuleCase:
    """Neo-Hookean capsules in simple shear between the walls."""
    name: str
    Lx: float
    Lz: float
    H: float
    alpha: float
    rc: float
    Nx: int
    Nz: int
    Ny: int
    nodes: np.ndarray        # (ncap * nv, 3) initial (pre-inflated) positions
    ref_nodes: np.ndarray    # (ncap * nv, 3) stress-free positions
    tri: np.ndarray          # (ncap * nf, 3) int32, outward orientation
    ncap: int
    nv: int
    a: float                 # radius after pre-inflation
    lam: float               # viscosity ratio
    ca: float                # capillary number mu shear a / G
    G: float                 # membrane shear modulus
    shear: float
    h_min: float             # minimum gap between surfaces (and to the walls)
    meta: dict


def case_capsule_suspension(ncap: int = 120, lam: float = 1.0, seed: int = 5, level: int = 2,
                            phi: float = 0.15, ca: float = 0.5) -> CapsuleCase:
    """Capsules of the suspension runs of Sec. 7.1: ncap spheres of 320
    triangles (level-2 icosphere, 162 nodes), pre-inflated by 5 % to radius
    a = 1, volume fraction phi in a cubic slit (Lx = Lz = 2H), simple shear
    of rate 1 at Ca = 0.5 (G = 2), r_c = a = 4/alpha, mean mesh spacing
    0.5/alpha in every direction (Nx = Nz the smallest even 2^a 3^b 5^c
    >= L/0.125, Ny - 1 = ceil(2H/0.125)), minimum gap 0.05 a.

    Draw order: the centres by random sequential addition (``_place_spheres``
    with centre distance >= 2.1 a and |y_c| <= H - 1.1 a), nothing else."""
    a, G, shear = 1.0, 1.0 / ca, 1.0
    L = (ncap * 4.0 * math.pi / 3.0 / phi) ** (1.0 / 3.0)
    H = 0.5 * L
    alpha = 4.0
    dx = 0.5 / alpha
    N = smooth_nodes(L, dx)
    Ny = int(math.ceil(2 * H / dx - 1e-12)) + 1
    rng = np.random.default_rng(seed)
    cen = _place_spheres(rng, ncap, L, H - 1.1 * a, 2.1 * a)
    V, F = icosphere(level)
    nodes = (cen[:, None, :] + a * V[None]).reshape(-1, 3)
    ref = (cen[:, None, :] + (a / 1.05) * V[None]).reshape(-1, 3)
    tri = (F[None] + (np.arange(ncap) * V.shape[0])[:, None, None]).reshape(-1, 3)
    return CapsuleCase(f"capsules_nh_{ncap}x{V.shape[0]}_lam{lam:g}", L, L, H, alpha, 1.0, N, N, Ny,
                       nodes, ref, tri.astype(np.int32), ncap, V.shape[0], a, float(lam), ca, G,
                       shear, 0.05 * a, dict(seed=seed, level=level, phi=phi))
