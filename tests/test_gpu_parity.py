"""Parity of the HIP path with the FP64 oracle, called through the C-ABI.

FP64 mode: relative max-norm error <= 1e-10 per output array (the oracle
solves the tau systems densely, the library by the even/odd recurrence; both
are backward stable and agree to ~1e-15 per mode).  Mixed mode: relative
2-norm error <= 1e-5 per output array.
"""
import numpy as np
import pytest

import oracle as O
from workloads import case_small_sl, random_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_1109_6587_amd as G  # noqa: E402

DEV = torch.device("cuda:0")
TOL64 = 1e-10
TOLMIX = 1e-5


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c0():
    c = case_small_sl(0)
    g = O.SlitGrid.from_case(c)
    ref = {
        "all": O.single_layer(g, c.xs, c.f, c.xt),
        "local": O.single_layer(g, c.xs, c.f, c.xt, parts=O.LOCAL),
        "global": O.single_layer(g, c.xs, c.f, c.xt, parts=O.GLOBAL),
        "spread": O.spread(g, g.wrap(c.xs), c.f),
    }
    return c, g, ref


def test_spread_grid_fp64(c0):
    c, g, ref = c0
    print(f"case {c.name} spread", flush=True)
    plan = G.Plan.from_case(c)
    F = plan.spread_grid(dev(c.xs), dev(c.f)).cpu().numpy()
    assert rel_max(F, ref["spread"]) < 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_spread_grid_coarse(precision, tol):
    """A coarse grid (dx = 2.5 r_c) whose tiles reach more than 64 rows of
    cells, so the spread describes them in two chunks of lanes; sources also
    outside [0, L) in x and z."""
    c = random_case(63, 300, 10, 40.0, 12.0, 2.0, 2.0, 8, 8, 9)   # mid tiles: 10 x 7 rows
    c.xs[::4, 0] -= 40.0
    c.xs[1::4, 2] += 80.0
    print(f"case {c.name} coarse spread {precision}", flush=True)
    g = O.SlitGrid.from_case(c)
    ref = O.spread(g, g.wrap(c.xs), c.f)
    plan = G.Plan.from_case(c, precision=precision)
    F = plan.spread_grid(dev(c.xs), dev(c.f)).cpu().numpy()
    assert rel_max(F, ref) < tol


@pytest.mark.parametrize("part", ["local", "global", "all"])
def test_single_layer_fp64(c0, part):
    c, g, ref = c0
    print(f"case {c.name} single layer fp64 part={part}", flush=True)
    parts = {"local": G.PART_LOCAL, "global": G.PART_GLOBAL, "all": G.PART_ALL}[part]
    plan = G.Plan.from_case(c)
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt), parts=parts).cpu().numpy()
    assert rel_max(u, ref[part]) < TOL64


def test_single_layer_mixed(c0):
    c, g, ref = c0
    print(f"case {c.name} single layer mixed", flush=True)
    plan = G.Plan.from_case(c, precision="mixed")
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    assert rel_l2(u, ref["all"]) < TOLMIX


def test_repeat_is_bitwise(c0):
    c, g, ref = c0
    plan = G.Plan.from_case(c)
    a = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    b = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    assert np.array_equal(a, b)


DL_CASES = [
    # seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz
    (11, 40, 70, 4.0, 1.0, 4.0, 1.5, 40, 32, 33, 3.5),
    (12, 150, 33, 6.0, 1.3, 3.0, 1.9, 48, 60, 25, None),
    (14, 60, 45, 4.0, 1.5, 3.0, 1.3, 20, 16, 65, None),      # Chebyshev order 64
    (15, 50, 30, 4.0, 1.5, 3.0, 1.3, 16, 16, 97, None),      # order above 64
]


@pytest.mark.parametrize("cfg", DL_CASES)
def test_double_layer_fp64(cfg):
    seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz = cfg
    c = random_case(seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz=Lz, dl=True)
    print(f"case {c.name} double layer fp64", flush=True)
    g = O.SlitGrid.from_case(c)
    ref = O.double_layer(g, c.xs, c.f, c.xt, c.normals)
    plan = G.Plan.from_case(c)
    v = plan.double_layer(dev(c.xs), dev(c.f), dev(c.xt), dev(c.normals)).cpu().numpy()
    for part, p in (("local", G.PART_LOCAL), ("global", G.PART_GLOBAL)):
        vp = plan.double_layer(dev(c.xs), dev(c.f), dev(c.xt), dev(c.normals), parts=p).cpu().numpy()
        refp = O.double_layer(g, c.xs, c.f, c.xt, c.normals, parts={"local": O.LOCAL, "global": O.GLOBAL}[part])
        assert rel_max(vp, refp) < TOL64, part
    assert rel_max(v, ref) < TOL64


SL_CASES = [
    (21, 1, 5, 4.0, 1.0, 4.0, 1.5, 32, 32, 17, None),       # one source
    (22, 300, 257, 5.0, 2.0, 2.5, 2.0, 40, 36, 33, 6.0),     # ragged, non-square box
    (23, 129, 3, 3.2, 0.7, 5.0, 1.2, 30, 50, 9, 3.0),       # radix 3/5 sizes, small Ny
    (24, 200, 90, 5.0, 2.0, 2.5, 1.6, 24, 24, 65, None),     # Chebyshev order 64
    (25, 80, 60, 4.0, 1.6, 3.0, 1.3, 16, 20, 97, None),      # order above 64
    (26, 40, 30, 4.0, 1.5, 3.0, 1.3, 16, 16, 129, None),     # largest order
]


@pytest.mark.parametrize("cfg", SL_CASES)
def test_single_layer_random_fp64(cfg):
    seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz = cfg
    c = random_case(seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz=Lz)
    print(f"case {c.name} single layer random fp64", flush=True)
    g = O.SlitGrid.from_case(c)
    ref = O.single_layer(g, c.xs, c.f, c.xt)
    plan = G.Plan.from_case(c)
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    assert rel_max(u, ref) < TOL64


@pytest.mark.parametrize("scale", [1.5, 2.0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cell_scale_keeps_the_result(scale, precision):
    """Larger cells (ggem_params.cell_scale) change only how the pairs are
    found: single and double layer still match the oracle (1e-10 FP64,
    1e-5 mixed), on a box with six cells across at the default size."""
    c = random_case(51, 400, 150, 12.0, 1.5, 2.0, 2.0, 48, 48, 33, dl=True)
    print(f"case {c.name} cell scale {scale} {precision}", flush=True)
    g = O.SlitGrid.from_case(c)
    ref_s = O.single_layer(g, c.xs, c.f, c.xt)
    ref_d = O.double_layer(g, c.xs, c.f, c.xt, c.normals)
    plan = G.Plan.from_case(c, precision=precision, cell_scale=scale)
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    v = plan.double_layer(dev(c.xs), dev(c.f), dev(c.xt), dev(c.normals)).cpu().numpy()
    if precision == "fp64":
        assert rel_max(u, ref_s) < TOL64 and rel_max(v, ref_d) < TOL64
    else:
        assert rel_l2(u, ref_s) < TOLMIX and rel_l2(v, ref_d) < TOLMIX


@pytest.mark.parametrize("Ny", [77, 121, 129])
def test_high_order_tau_mixed(Ny):
    """Chebyshev orders above 64 in mixed precision (the register sweeps up to
    order 128, the LDS form above): single and double layer against the
    oracle (1e-5)."""
    c = random_case(62, 60, 40, 4.0, 1.5, 3.0, 1.3, 16, 16, Ny, dl=True)
    print(f"case {c.name} Ny={Ny} mixed", flush=True)
    g = O.SlitGrid.from_case(c)
    ref_s = O.single_layer(g, c.xs, c.f, c.xt)
    ref_d = O.double_layer(g, c.xs, c.f, c.xt, c.normals)
    plan = G.Plan.from_case(c, precision="mixed")
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    v = plan.double_layer(dev(c.xs), dev(c.f), dev(c.xt), dev(c.normals)).cpu().numpy()
    assert rel_l2(u, ref_s) < TOLMIX and rel_l2(v, ref_d) < TOLMIX


def test_empty_inputs():
    c = random_case(31, 10, 10, 4.0, 1.0, 4.0, 1.0, 16, 16, 9)
    plan = G.Plan.from_case(c)
    xs0 = torch.zeros((0, 3), dtype=torch.float64, device=DEV)
    u = plan.single_layer(xs0, xs0, dev(c.xt)).cpu().numpy()
    assert np.all(u == 0.0)
    out = plan.single_layer(dev(c.xs), dev(c.f), xs0)
    assert out.shape == (0, 3)


MIXED_MODES = ["mixed", "mixed_bf16"]   # FP32 MFMA / BF16 hi+lo split Chebyshev products


@pytest.mark.parametrize("precision", MIXED_MODES)
@pytest.mark.parametrize("cfg", DL_CASES + [(13, 300, 100, 5.0, 1.5, 2.0, 2.0, 40, 40, 33, None)])
def test_double_layer_mixed(cfg, precision):
    seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz = cfg
    c = random_case(seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz=Lz, dl=True)
    print(f"case {c.name} double layer {precision}", flush=True)
    g = O.SlitGrid.from_case(c)
    ref = O.double_layer(g, c.xs, c.f, c.xt, c.normals)
    plan = G.Plan.from_case(c, precision=precision)
    v = plan.double_layer(dev(c.xs), dev(c.f), dev(c.xt), dev(c.normals)).cpu().numpy()
    assert rel_l2(v, ref) < TOLMIX


@pytest.mark.parametrize("precision", MIXED_MODES)
@pytest.mark.parametrize("cfg", SL_CASES)
def test_single_layer_random_mixed(cfg, precision):
    seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz = cfg
    c = random_case(seed, ns, nt, L, H, alpha, rc, Nx, Nz, Ny, Lz=Lz)
    print(f"case {c.name} single layer random {precision}", flush=True)
    g = O.SlitGrid.from_case(c)
    ref = O.single_layer(g, c.xs, c.f, c.xt)
    plan = G.Plan.from_case(c, precision=precision)
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
    assert rel_l2(u, ref) < TOLMIX


@pytest.mark.parametrize("precision", MIXED_MODES)
def test_global_part_mixed(c0, precision):
    """The global part alone (where the Chebyshev products act), against the
    oracle's global part."""
    c, g, ref = c0
    print(f"case {c.name} global part {precision}", flush=True)
    plan = G.Plan.from_case(c, precision=precision)
    u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt), parts=G.PART_GLOBAL).cpu().numpy()
    assert rel_l2(u, ref["global"]) < TOLMIX
