"""Edge cases of the HIP path against the FP64 oracle, through the C ABI.

* Positions outside [0, L) in x and z (negative, equal to L, several periods
  away), as a time-stepped suspension produces them: the library wraps them
  as the oracle does.
* Targets exactly on the walls y = -H and y = +H (on and off the mesh).
* Duplicate sources (identical positions) and near-coincident points: points
  closer than one FP32 rounding of their cell-relative coordinates must still
  be an ordinary pair in mixed precision, and only exactly coincident points
  take the self rule.
* Domain and capacity errors of a single plan (non-finite input, a source on
  or beyond a wall, a target beyond a wall, more points than reserved), both
  with synchronous checks and through ggem_plan_status, and the plan still
  evaluates correctly afterwards.

FP64 to 1e-10 (relative max-norm), mixed precision to 1e-5 (relative 2-norm).
"""
import numpy as np
import pytest

import oracle as O
from workloads import random_case

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


def check(got, ref, precision):
    if precision == "fp64":
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        assert err < TOL64, err
    else:
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        assert err < TOLMIX, err


def run(c, xs, f, xt, nrm, precision):
    plan = G.Plan.from_case(c, precision=precision, max_src=len(xs), max_tgt=len(xt))
    if nrm is None:
        out = plan.single_layer(dev(xs), dev(f), dev(xt))
    else:
        out = plan.double_layer(dev(xs), dev(f), dev(xt), dev(nrm))
    res = out.cpu().numpy()
    plan.close()
    return res


def oracle_eval(c, xs, f, xt, nrm):
    g = O.SlitGrid.from_case(c)
    if nrm is None:
        return O.single_layer(g, xs, f, xt)
    return O.double_layer(g, xs, f, xt, nrm)


def unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("layer", ["single", "double"])
def test_unwrapped_positions(precision, layer):
    c = random_case(41, 300, 200, 8.0, 1.0, 3.0, 4.0 / 3.0, 32, 32, 25)
    rng = np.random.default_rng(41)
    xs, xt = c.xs.copy(), c.xt.copy()
    for a in (xs, xt):
        a[:, 0] += c.Lx * rng.integers(-3, 4, len(a))
        a[:, 2] += c.Lz * rng.integers(-3, 4, len(a))
    xs[:4, 0] = [0.0, c.Lx, -c.Lx, 2 * c.Lx]      # exact multiples of the period
    # the targets that are sources move with them (a point of a time-stepped
    # surface is one position, however far it has travelled)
    xt[:c.ns] = xs
    xt[-3:, 2] = [c.Lz, -c.Lz, 0.0]
    nrm = unit(rng, len(xt)) if layer == "double" else None
    print(f"unwrapped {layer} {precision}: {len(xs)} sources, {len(xt)} targets", flush=True)
    check(run(c, xs, c.f, xt, nrm, precision), oracle_eval(c, xs, c.f, xt, nrm), precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("layer", ["single", "double"])
def test_targets_on_the_walls(precision, layer):
    c = random_case(42, 250, 0, 8.0, 1.0, 3.0, 4.0 / 3.0, 32, 32, 25,
                    include_sources_as_targets=False)
    rng = np.random.default_rng(42)
    m = 60
    on_mesh = np.stack([rng.integers(0, 32, m) * c.Lx / 32, np.where(np.arange(m) % 2, c.H, -c.H),
                        rng.integers(0, 32, m) * c.Lz / 32], 1)
    off_mesh = np.stack([rng.uniform(0, c.Lx, m), np.where(np.arange(m) % 2, -c.H, c.H),
                         rng.uniform(0, c.Lz, m)], 1)
    xt = np.vstack([on_mesh, off_mesh, c.xs[:40]])
    nrm = unit(rng, len(xt)) if layer == "double" else None
    print(f"wall targets {layer} {precision}: {len(xt)} targets", flush=True)
    check(run(c, c.xs, c.f, xt, nrm, precision), oracle_eval(c, c.xs, c.f, xt, nrm), precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("layer", ["single", "double"])
def test_duplicate_and_near_coincident_points(precision, layer):
    c = random_case(43, 200, 100, 8.0, 1.0, 3.0, 4.0 / 3.0, 32, 32, 25)
    rng = np.random.default_rng(43)
    xs, f = c.xs.copy(), c.f.copy()
    # exact duplicates of ten sources (different strengths)
    dup = xs[:10].copy()
    # near-coincident copies: 2e-8 (below one FP32 rounding of a coordinate),
    # 1e-13 (where FP32 intermediates of the kernels would overflow) and 0.02
    # (an ordinary FP32 pair; the FP64 path takes alpha r < 0.01)
    near = np.vstack([xs[10:20], xs[20:30], xs[30:40]])
    off = np.repeat([2e-8, 1e-13, 0.02], 10)[:, None]
    near[:, [0]] += off
    near[:, [2]] -= off
    xs = np.vstack([xs, dup, near])
    f = np.vstack([f, rng.standard_normal((40, 3))])
    # targets: the originals (coincident with the duplicates) and the probes
    xt = c.xt
    nrm = unit(rng, len(xt)) if layer == "double" else None
    print(f"duplicates {layer} {precision}: {len(xs)} sources, {len(xt)} targets", flush=True)
    check(run(c, xs, f, xt, nrm, precision), oracle_eval(c, xs, f, xt, nrm), precision)


def test_single_plan_errors():
    c = random_case(44, 100, 50, 8.0, 1.0, 3.0, 4.0 / 3.0, 32, 32, 25)
    print("single-plan error codes", flush=True)
    ref = oracle_eval(c, c.xs, c.f, c.xt, None)
    for sync in (True, False):
        plan = G.Plan.from_case(c, max_src=c.ns, max_tgt=c.nt, sync_checks=sync)
        bad = []
        xs = c.xs.copy()
        xs[7, 1] = np.nan
        bad.append((xs, c.xt))
        xs = c.xs.copy()
        xs[3, 1] = c.H                      # a source on the wall
        bad.append((xs, c.xt))
        xs = c.xs.copy()
        xs[5, 1] = -1.5 * c.H
        bad.append((xs, c.xt))
        xt = c.xt.copy()
        xt[9, 1] = c.H * (1 + 1e-12)        # a target beyond the wall
        bad.append((c.xs, xt))
        xt = c.xt.copy()
        xt[2, 0] = np.inf
        bad.append((c.xs, xt))
        for xs, xt in bad:
            with pytest.raises(G.GGEMError) as e:
                plan.single_layer(dev(xs), dev(c.f), dev(xt))
                plan.status()
            assert e.value.code == G.ggem.E_DOMAIN
        # too many points for the plan's capacities: refused before any device work
        with pytest.raises(G.GGEMError) as e:
            plan.single_layer(dev(np.vstack([c.xs, c.xs[:1]])), dev(np.vstack([c.f, c.f[:1]])),
                              dev(c.xt))
        assert e.value.code == G.ggem.E_CAPACITY
        with pytest.raises(G.GGEMError) as e:
            plan.single_layer(dev(c.xs), dev(c.f), dev(np.vstack([c.xt, c.xt[:1]])))
        assert e.value.code == G.ggem.E_CAPACITY
        # the plan still evaluates correctly after the errors
        u = plan.single_layer(dev(c.xs), dev(c.f), dev(c.xt)).cpu().numpy()
        plan.status()
        check(u, ref, "fp64")
        plan.close()
