"""Spectrally accurate off-mesh evaluation (GGEM_INTERP_SPECTRAL) through the
C-ABI, against the direct Fourier-Chebyshev series of oracle/spectral.py
(Sec. 3.2.2, last paragraph: the non-uniform FFT keeps the spectral accuracy
of the mesh points at any point)."""
import numpy as np
import pytest

import oracle as O
import oracle.spectral as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402

DEV = torch.device("cuda:0")
MSP = {"fp64": 12, "mixed": 6}
TOL = {"fp64": 1e-10, "mixed": 1e-5}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def plan_for(g, precision, ns, nt, msp):
    p = G.Plan(g.Lx, g.Lz, g.H, g.alpha, g.Nx, g.Nz, g.Ny, rc=g.rc, precision=precision,
               max_src=ns, max_tgt=nt)
    p.set_interp(G.INTERP_SPECTRAL, msp)
    return p


@pytest.fixture(scope="module")
def small():
    """Lx != Lz and Nx != Nz (radices 2, 5 and 2, 3), targets coincident with
    sources, on both walls, at other periodic images, and one more than a
    256-wide block (ragged tail)."""
    rng = np.random.default_rng(41)
    Lx, Lz, H, alpha = 3.0, 2.4, 1.0, 4.0
    g = O.SlitGrid(Lx, Lz, H, alpha, 1.0, 40, 24, 33)
    ns, nt = 60, 257
    xs = np.stack([rng.uniform(0, Lx, ns), rng.uniform(-0.95, 0.95, ns), rng.uniform(0, Lz, ns)], 1)
    f = rng.standard_normal((ns, 3))
    xt = np.stack([rng.uniform(0, Lx, nt), rng.uniform(-H, H, nt), rng.uniform(0, Lz, nt)], 1)
    xt[:4] = xs[:4]
    xt[4, 1], xt[5, 1] = H, -H
    xt[6] += [-Lx, 0.0, 2 * Lz]
    xt[7] += [2 * Lx, 0.0, -Lz]
    nrm = unit(rng, nt)
    return g, xs, f, xt, nrm, S.single_layer_spectral(g, xs, f, xt), \
        S.double_layer_spectral(g, xs, f, xt, nrm)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_spectral_parity_small(small, precision):
    g, xs, f, xt, nrm, ref_s, ref_d = small
    print(f"spectral small {precision}", flush=True)
    p = plan_for(g, precision, len(xs), len(xt), MSP[precision])
    u = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
    assert np.abs(u - ref_s).max() < TOL[precision] * np.abs(ref_s).max()
    v = p.double_layer(dev(xs), dev(f), dev(xt), dev(nrm)).cpu().numpy()
    assert np.abs(v - ref_d).max() < TOL[precision] * np.abs(ref_d).max()
    # a second, smaller call on the same plan
    u2 = p.single_layer(dev(xs[:20]), dev(f[:20]), dev(xt[:9])).cpu().numpy()
    ref2 = S.single_layer_spectral(g, xs[:20], f[:20], xt[:9])
    assert np.abs(u2 - ref2).max() < TOL[precision] * np.abs(ref2).max()
    p.close()


def test_targets_are_the_sources(small):
    """Coinciding targets reuse the sources' binning (the surface case)."""
    g, xs, f, _, _, _, _ = small
    rng = np.random.default_rng(8)
    nrm = unit(rng, len(xs))
    p = plan_for(g, "fp64", len(xs), len(xs), 12)
    xs_d = dev(xs)
    u = p.single_layer(xs_d, dev(f), xs_d).cpu().numpy()
    ref = S.single_layer_spectral(g, xs, f, xs)
    assert np.abs(u - ref).max() < 1e-10 * np.abs(ref).max()
    v = p.double_layer(xs_d, dev(f), xs_d, dev(nrm)).cpu().numpy()
    ref = S.double_layer_spectral(g, xs, f, xs, nrm)
    assert np.abs(v - ref).max() < 1e-10 * np.abs(ref).max()
    p.close()


def test_parts_and_empty(small):
    g, xs, f, xt, _, ref_s, _ = small
    p = plan_for(g, "fp64", len(xs), len(xt), 12)
    ul = p.single_layer(dev(xs), dev(f), dev(xt), parts=G.PART_LOCAL).cpu().numpy()
    ug = p.single_layer(dev(xs), dev(f), dev(xt), parts=G.PART_GLOBAL).cpu().numpy()
    assert np.abs(ul + ug - ref_s).max() < 1e-10 * np.abs(ref_s).max()
    gw, xw = g.wrap(xs), g.wrap(xt)
    loc = O.local_velocity(g, gw, f, xw)
    assert np.abs(ul - loc).max() < 1e-12 * np.abs(loc).max()
    # no targets; no sources (the global part of nothing is zero)
    assert p.single_layer(dev(xs), dev(f), dev(xt[:0])).shape[0] == 0
    z = p.single_layer(dev(xs[:0]), dev(f[:0]), dev(xt)).cpu().numpy()
    assert np.abs(z).max() == 0.0
    p.close()


def test_mode_switch_and_errors(small):
    g, xs, f, xt, _, ref_s, _ = small
    p = plan_for(g, "fp64", len(xs), len(xt), 12)
    us = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
    p.set_interp(G.INTERP_LAGRANGE)
    ul = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
    ref_l = O.single_layer(g, xs, f, xt)
    assert np.abs(ul - ref_l).max() < 1e-10 * np.abs(ref_l).max()
    # the two differ off the mesh by the stencil's O(h^5) error only
    assert np.abs(us - ul).max() < 1e-2 * np.abs(ref_s).max()
    for mode, msp in ((2, 12), (G.INTERP_SPECTRAL, 1), (G.INTERP_SPECTRAL, 17),
                      (G.INTERP_SPECTRAL, 25)):
        with pytest.raises(G.GGEMError) as e:
            p.set_interp(mode, msp)
        assert e.value.code == G.ggem.E_ARG
    p.close()
    big = G.Plan(4.0, 4.0, 1.0, 4.0, 320, 16, 9, rc=1.0, max_src=1, max_tgt=1)
    with pytest.raises(G.GGEMError) as e:
        big.set_interp(G.INTERP_SPECTRAL, 8)
    assert e.value.code == G.ggem.E_ARG
    big.close()


def test_spectral_convergence_off_the_mesh():
    """The paper's convergence experiment (its Fig. on an off-mesh target):
    point force (F, F, F) at (L/4, -H/2, L/4), target (0.4312 L,
    0.3734 (2H) - H, 0.5234 L), L = 4H, alpha = 4, r_c = 6/alpha.  Against
    the series on a 64 x 64 x 65 grid the spectral evaluation is below 1e-8
    at 48 points per period where the Lagrange stencil is above 1e-7."""
    H, L, alpha = 1.0, 4.0, 4.0
    xs = np.array([[0.25 * L, -0.5 * H, 0.25 * L]])
    f = np.ones((1, 3))
    xt = np.array([[0.4312 * L, 0.3734 * 2 * H - H, 0.5234 * L]])
    ref = S.single_layer_spectral(O.SlitGrid(L, L, H, alpha, 6.0 / alpha, 64, 64, 65), xs, f, xt)
    g = O.SlitGrid(L, L, H, alpha, 6.0 / alpha, 48, 48, 49)
    p = plan_for(g, "fp64", 1, 1, 12)
    us = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
    p.set_interp(G.INTERP_LAGRANGE)
    ul = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
    scale = np.abs(ref).max()
    print(np.abs(us - ref).max() / scale, np.abs(ul - ref).max() / scale)
    assert np.abs(us - ref).max() < 1e-8 * scale
    assert np.abs(ul - ref).max() > 1e-7 * scale
    p.close()


@pytest.fixture(scope="module")
def medium():
    rng = np.random.default_rng(43)
    L, H, N, Ny, alpha = 3.2, 1.2, 64, 65, 5.0
    g = O.SlitGrid(L, L, H, alpha, 4.0 / alpha, N, N, Ny)
    ns = 2000
    xs = np.stack([rng.uniform(0, L, ns), rng.uniform(-1.15, 1.15, ns), rng.uniform(0, L, ns)], 1)
    f = rng.standard_normal((ns, 3))
    xt = np.stack([rng.uniform(0, L, 16), rng.uniform(-H, H, 16), rng.uniform(0, L, 16)], 1)
    return g, xs, f, xt, S.single_layer_spectral(g, xs, f, xt)


def test_spectral_parity_medium(medium):
    """2000 sources on a 64 x 64 x 65 grid (many spread tiles), 16 sampled
    targets against the series; the mesh nodes against the Lagrange path,
    which reproduces the grid values there."""
    g, xs, f, xt, ref = medium
    p = plan_for(g, "fp64", len(xs), 4096, 12)
    u = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
    assert np.abs(u - ref).max() < 1e-10 * np.abs(ref).max()
    rng = np.random.default_rng(9)
    i, j, k = rng.integers(0, 64, 4096), rng.integers(0, 65, 4096), rng.integers(0, 64, 4096)
    nodes = np.stack([g.x[i], g.y[j], g.z[k]], 1)
    us = p.single_layer(dev(xs), dev(f), dev(nodes)).cpu().numpy()
    p.set_interp(G.INTERP_LAGRANGE)
    ul = p.single_layer(dev(xs), dev(f), dev(nodes)).cpu().numpy()
    assert np.abs(us - ul).max() < 1e-10 * np.abs(ul).max()
    p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("grid", [(40, 24, 33), (32, 32, 65)])
def test_window_width_error_law(precision, grid):
    """Every window width the kernels specialise for (FP64: 1, 2, 4, 9 and 16
    entries per lane; FP32: 2, 4, 8 and 16 vectors per lane and row) has the
    error of Gaussian gridding with oversampling 2, below exp(-0.75 pi msp)
    of the largest value, down to the rounding floor of the grid's type."""
    Nx, Nz, Ny = grid
    rng = np.random.default_rng(41)
    Lx, Lz, H, alpha = 3.0, 2.4, 1.0, 4.0
    g = O.SlitGrid(Lx, Lz, H, alpha, 1.0, Nx, Nz, Ny)
    ns, nt = 60, 257
    xs = np.stack([rng.uniform(0, Lx, ns), rng.uniform(-0.95, 0.95, ns), rng.uniform(0, Lz, ns)], 1)
    f = rng.standard_normal((ns, 3))
    xt = np.stack([rng.uniform(0, Lx, nt), rng.uniform(-H, H, nt), rng.uniform(0, Lz, nt)], 1)
    nrm = unit(rng, nt)
    ref = S.single_layer_spectral(g, xs, f, xt)
    refd = S.double_layer_spectral(g, xs, f, xt, nrm)
    floor = 1e-13 if precision == "fp64" else 1e-6
    for msp in (2, 4, 5, 8, 10, 16):
        print(f"grid {grid} {precision} msp {msp}", flush=True)
        bound = np.exp(-0.75 * np.pi * msp) + floor
        p = plan_for(g, precision, ns, nt, msp)
        u = p.single_layer(dev(xs), dev(f), dev(xt)).cpu().numpy()
        v = p.double_layer(dev(xs), dev(f), dev(xt), dev(nrm)).cpu().numpy()
        assert np.abs(u - ref).max() < bound * np.abs(ref).max(), msp
        assert np.abs(v - refd).max() < bound * np.abs(refd).max(), msp
        p.close()
