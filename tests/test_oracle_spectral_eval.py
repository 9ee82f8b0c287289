"""Pins of the spectral off-mesh evaluation (oracle/spectral.py): it is the
grid value at mesh nodes, and off the mesh it converges spectrally where the
4th-order Lagrange stencil stops at its O(h^5) error (Sec. 3.2.2, last
paragraph; the paper's convergence experiment, Sec. 3.2.3)."""
import numpy as np

import oracle as O
import oracle.spectral as S


def test_series_equals_the_grid_at_mesh_nodes():
    rng = np.random.default_rng(1)
    g = O.SlitGrid(2.0, 2.0, 0.75, 8.0, 0.75, 32, 32, 33)
    xs = np.stack([rng.uniform(0, 2, 10), rng.uniform(-0.6, 0.6, 10), rng.uniform(0, 2, 10)], 1)
    f = rng.standard_normal((10, 3))
    j, i, k = rng.integers(0, 33, 8), rng.integers(0, 32, 8), rng.integers(0, 32, 8)
    xt = np.stack([g.x[i], g.y[j], g.z[k]], 1)
    ref = O.single_layer(g, xs, f, xt)
    assert np.abs(S.single_layer_spectral(g, xs, f, xt) - ref).max() < 1e-13 * np.abs(ref).max()
    nrm = rng.standard_normal((8, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ref = O.double_layer(g, xs, f, xt, nrm)
    got = S.double_layer_spectral(g, xs, f, xt, nrm)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_spectral_convergence_off_the_mesh():
    """One point force (F, F, F) at (L/4, -H/2, L/4), the off-mesh target
    (0.4312 L, 0.3734 (2H) - H, 0.5234 L) of the paper's convergence test
    (its y in [0, 2H] shifted by -H), here with L = 4H, alpha = 4 and
    r_c = 6/alpha.  Against the series on a 64 x 64 x 65 grid, the series
    error falls by more than 1e3 from 32 to 48 points per period and is
    below 1e-8 there, while the Lagrange stencil is still above 1e-7."""
    H, L, alpha = 1.0, 4.0, 4.0
    xs = np.array([[0.25 * L, -0.5 * H, 0.25 * L]])
    f = np.ones((1, 3))
    xt = np.array([[0.4312 * L, 0.3734 * 2 * H - H, 0.5234 * L]])

    def run(N, spectral):
        g = O.SlitGrid(L, L, H, alpha, 6.0 / alpha, N, N, N + 1)
        return (S.single_layer_spectral if spectral else O.single_layer)(g, xs, f, xt)

    ref = run(64, True)
    scale = np.abs(ref).max()
    err_s = {N: np.abs(run(N, True) - ref).max() / scale for N in (32, 48)}
    err_l = np.abs(run(48, False) - ref).max() / scale
    print(err_s, err_l)
    assert err_s[48] < 1e-8 and err_l > 1e-7
    assert err_s[48] < 1e-3 * err_s[32]
