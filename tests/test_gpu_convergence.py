"""The convergence experiment of Sec. 3.2.3 (Fig. ggem_conv) through the
C-ABI, FP64: a point force (F, F, F) at (L/4, L/4, L/4) of a slit with
L_x = L_z = wall spacing = L, alpha = 80/(3L), observed at the mesh point
(L/2, L/2, L/2) and the off-mesh point (0.4312, 0.3734, 0.5234) L (the
paper's frame, y from the lower wall); reference N_y = 129, r_c = 13/alpha.
The paper reports an error of O(1e-6) on the mesh at r_c = 4/alpha, a
plateau set by r_c, and an h^5 floor off the mesh from the Lagrange stencil,
which the spectral evaluation removes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402

DEV = torch.device("cuda:0")
L, ALPHA = 1.0, 80.0 / 3.0


def ux(Ny, C, spectral):
    H = 0.5 * L
    xs = torch.tensor([[0.25 * L, 0.25 * L - H, 0.25 * L]], dtype=torch.float64, device=DEV)
    f = torch.ones((1, 3), dtype=torch.float64, device=DEV)
    xt = torch.tensor([[0.5 * L, 0.5 * L - H, 0.5 * L], [0.4312 * L, 0.3734 * L - H, 0.5234 * L]],
                      dtype=torch.float64, device=DEV)
    p = G.Plan(L, L, H, ALPHA, Ny - 1, Ny - 1, Ny, rc=C / ALPHA, precision="fp64", max_src=1,
               max_tgt=2)
    if spectral:
        p.set_interp(G.INTERP_SPECTRAL, 12)
    u = p.single_layer(xs, f, xt).cpu().numpy()[:, 0]
    p.close()
    return u


@pytest.fixture(scope="module")
def ref():
    return ux(129, 13.0, True)


def rel(a, b):
    return np.abs(a - b) / np.abs(b)


def test_mesh_point_plateau_set_by_rc(ref):
    """At (alpha dy)^-1 = 4.5 the mesh-point error has reached the plateau of
    its r_c: O(1e-6) for r_c = 4/alpha, far lower for 5/alpha and 6/alpha."""
    e4 = rel(ux(121, 4.0, False), ref)[0]
    e6 = rel(ux(121, 6.0, False), ref)[0]
    print(e4, e6)
    assert 1e-6 < e4 < 3e-5
    assert e6 < 1e-11


def test_off_mesh_floor_and_its_removal(ref):
    """r_c = 6/alpha: off the mesh the Lagrange stencil's error falls
    algebraically (about h^5 between N_y = 65 and 121) and stays above 1e-8,
    while the spectral evaluation follows the mesh-point convergence."""
    l65, l121 = rel(ux(65, 6.0, False), ref)[1], rel(ux(121, 6.0, False), ref)[1]
    s121 = rel(ux(121, 6.0, True), ref)[1]
    print(l65, l121, s121)
    assert l121 > 1e-8
    assert 10 < l65 / l121 < 100          # (120/64)^5 = 23
    assert s121 < 1e-11
