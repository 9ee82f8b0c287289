"""Mutation check of the oracle's pins (CPU).

Each case plants one plausible mistake in a copy of an oracle module (a
sign, a dropped term, a transposed operand, a wrong index, a missing 1/H, a
wrong scale factor), swaps the copy in for the oracle, and runs the pins of
tests/test_oracle_*.py against it: at least one must fail.  The unmutated oracle passes the same
checks (control), so a failure is the mutation's doing.
"""
import types

import numpy as np
import pytest

import oracle
import oracle.bi
import oracle.capsule
import oracle.fredholm
import oracle.ggem
import oracle.probes
import oracle.surface
import test_oracle_bi as BI
import test_oracle_capsule as CAP
import test_oracle_invariants as INV
import test_oracle_kernels as KER
import test_oracle_physics as PHY
import test_oracle_probes as PRB
import test_oracle_spectral as SPE

pytestmark = pytest.mark.slow

MUTATIONS = {
    "Fredholm operator scale (kappa instead of 2 kappa)": ("fredholm",
        "return x + 2.0 * k * v",
        "return x + k * v"),
    "surface velocity scale (4 pi instead of 8 pi)": ("surface",
        "u = 8.0 * np.pi * single_layer(",
        "u = 4.0 * np.pi * single_layer("),
    "pressure equation sign": ("ggem",
        "divF = ikx * fx + (fy @ D.T) / H + ikz * fz",
        "divF = -(ikx * fx + (fy @ D.T) / H + ikz * fz)"),
    "dropped pressure gauge": ("ggem",
        "gauge = pressure_gauge(g, xs, f) if stress else 0.0",
        "gauge = 0.0"),
    "dropped self term": ("ggem",
        "self_coef = -(4.0 * g.alpha / SQRT_PI) * INV_8PI",
        "self_coef = 0.0"),
    "transposed Chebyshev operand": ("ggem",
        'return np.einsum("nj,...jab->...nab", M, a)',
        'return np.einsum("jn,...jab->...nab", M, a)'),
    "wrong wavenumber in sigma_xy": ("ggem",
        "dy(u) + ikx * v,",
        "dy(u) + ikz * v,"),
    "dropped Gaussian term of G^l": ("ggem",
        "- (2.0 * alpha / SQRT_PI) * (I - dd / r2[..., None, None]) * ex[..., None, None])",
        "- 0.0 * (I - dd / r2[..., None, None]) * ex[..., None, None])"),
    "wall data sign": ("ggem",
        "out.append(-ul.T.reshape(3, g.Nx, g.Nz))",
        "out.append(ul.T.reshape(3, g.Nx, g.Nz))"),
    "k = 0 pressure without 1/H": ("ggem",
        "A[:N] = D[:N] / H",
        "A[:N] = D[:N]"),
    "stresslet B term sign": ("ggem",
        "+ 4.0 * alpha ** 3 / SQRT_PI * (dI - 2.0 * ddd / e(r2)) * e(ex))",
        "- 4.0 * alpha ** 3 / SQRT_PI * (dI - 2.0 * ddd / e(r2)) * e(ex))"),
    "dropped (1 - eta) Jacobian of the parent triangle": ("bi",
        "wts.append(wi * wj * (1.0 - tj))",
        "wts.append(wi * wj)"),
    "dropped polar Jacobian rho": ("bi",
        "wts.append((0.5 * math.pi * wk) * (rmax * wi) * rho)",
        "wts.append((0.5 * math.pi * wk) * (rmax * wi))"),
    "n(z) kept on the element at z (no n~)": ("bi",
        "m = phi[:, :1] * nD + (1.0 - phi[:, :1]) * nz",
        "m = np.broadcast_to(nz, (len(wts), 3))"),
    "probe pressure without the gauge": ("probes",
        "dft_xz(g, gp), pressure_gauge(g, xs, f))",
        "dft_xz(g, gp), 0.0)"),
    "probe sigma_xy with the z wavenumber": ("probes",
        "dy(u) + ikx * v, ikz * u + ikx * w, ikz * v + dy(w))",
        "dy(u) + ikz * v, ikz * u + ikx * w, ikz * v + dy(w))"),
    "particle stress with lambda + 1": ("probes",
        "S += (lam - 1.0) * (",
        "S += (lam + 1.0) * ("),
    "torque row with r and f swapped": ("bi",
        "T = (A[:, None] * np.cross(r, f)).sum(axis=0)",
        "T = (A[:, None] * np.cross(f, r)).sum(axis=0)"),
    "principal-stretch derivative with swapped exponents": ("capsule",
        "dW = G * (lam - 1.0 / (lam ** 3 * lam[::-1] ** 2))",
        "dW = G * (lam - 1.0 / (lam ** 2 * lam[::-1] ** 3))"),
    "traction jump over the reference node areas": ("capsule",
        "return -F / node_areas(nodes, tri)[:, None], energy",
        "return -F / node_areas(ref_nodes, tri)[:, None], energy"),
    "membrane force left in the element's x direction": ("capsule",
        "np.outer(f2[:, 0], t1) + np.outer(f2[:, 1], t2)",
        "np.outer(f2[:, 0], t1) + np.outer(f2[:, 1], t1)"),
    "volume correction of the wrong sign": ("capsule",
        "out[sl] += (v0[c] - v[c]) / area[sl].sum() * normals[sl]",
        "out[sl] += (v[c] - v0[c]) / area[sl].sum() * normals[sl]"),
    "index of the Lagrange stencil in y": ("ggem",
        "wy = _lagrange(xt[:, 1], g.y[jj])",
        "wy = _lagrange(xt[:, 1], g.y[jj[:, ::-1]])"),
}


def mutant(module, old, new):
    with open(getattr(oracle, module).__file__) as fh:
        src = fh.read()
    assert src.count(old) == 1, old
    src = src.replace(old, new).replace("from .", "from oracle.")
    mod = types.ModuleType(f"oracle_{module}_mutant")
    exec(compile(src, f"oracle_{module}_mutant", "exec"), mod.__dict__)
    return mod


def install(monkeypatch, mod):
    """Point the oracle package (and the modules that import from it) at `mod`."""
    for name, val in vars(mod).items():
        if name.startswith("__") or not callable(val) and not isinstance(val, (int, float)):
            continue
        for target in (oracle.ggem, oracle, oracle.fredholm, oracle.surface, oracle.bi,
                       oracle.probes, oracle.capsule):
            if hasattr(target, name):
                monkeypatch.setattr(target, name, val)


def alpha_independence():
    """SL with self pairs and DL at mesh nodes, alpha 4 vs 5 (r_c = 6/alpha)."""
    rng = np.random.default_rng(5)
    L, H, N, Ny = 3.2, 1.2, 48, 65
    g0 = oracle.SlitGrid(L, L, H, 4.0, 1.5, N, N, Ny)
    xs = np.stack([rng.uniform(0, L, 4), rng.uniform(-0.8, 0.8, 4), rng.uniform(0, L, 4)], 1)
    xs[:2] = [[g0.x[9], g0.y[30], g0.z[40]], [g0.x[40], g0.y[20], g0.z[3]]]
    f = rng.standard_normal((4, 3))
    j, i, k = rng.integers(0, Ny, 20), rng.integers(0, N, 20), rng.integers(0, N, 20)
    xt = np.vstack([np.stack([g0.x[i], g0.y[j], g0.z[k]], 1), xs[:2]])
    nrm = rng.standard_normal(xt.shape)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    res = []
    for a in (4.0, 5.0):
        g = oracle.SlitGrid(L, L, H, a, 6.0 / a, N, N, Ny)
        res.append((oracle.single_layer(g, xs, f, xt), oracle.double_layer(g, xs, f, xt, nrm)))
    for q in range(2):
        a, b = res[0][q], res[1][q]
        assert np.abs(a - b).max() < 1e-8 * np.abs(a).max()


def bi_sphere():
    V, F = BI.icosphere(1)
    xc = np.array([1.0, 0.0, 1.0])
    return oracle.SlitGrid(2.0, 2.0, 0.75, 8.0, 0.5, 32, 32, 33), V * 0.3 + xc, F, xc


def probe_field():
    return PRB.field.__wrapped__()


def interpolation_of_polynomials():
    SPE.test_interpolation_reproduces_polynomials(np.random.default_rng(7))


# cheapest first: a mutant stops at the first pin that fails
CHECKS = [
    ("membrane forces are the energy gradient", CAP.test_forces_are_minus_the_energy_gradient),
    ("uniformly inflated capsule", CAP.test_uniform_inflation_is_a_uniform_tension),
    ("membrane rigid-motion invariance", CAP.test_rigid_motion_invariance),
    ("volume correction", CAP.test_volume_correction),
    ("G^l is Stokes flow", lambda: KER.test_local_pair_is_stokes_flow(0)),
    ("element rule on polynomials", BI.test_regular_rule_exact_for_polynomials),
    ("vertex element in closed form",
     lambda: BI.test_vertex_element_singular_integral(((0.3, 0.05, 0.0), (0.1, 0.25, 0.02)))),
    ("double-layer vertex element with n~", BI.test_dl_vertex_element_with_ntilde),
    ("T^l is the Newtonian stress", lambda: KER.test_stresslet_is_newtonian_stress(3)),
    ("manufactured Stokes mode", lambda: SPE.test_stokes_mode_manufactured((3, 1), np.random.default_rng(1))),
    ("manufactured zero mode", lambda: SPE.test_stokes_zero_mode_manufactured(np.random.default_rng(2))),
    ("Lagrange interpolation", interpolation_of_polynomials),
    ("no-slip", lambda: INV.test_no_slip_at_walls(np.random.default_rng(12345))),
    ("alpha independence", alpha_independence),
    ("wall force balance", PHY.test_wall_force_balance),
    ("Fredholm operator on q = n", PHY.test_fredholm_uniform_normal_density),
    ("surface velocity of a uniform density", PHY.test_surface_velocity_uniform_density_translates_sphere),
    ("torque of a rotational traction", lambda: BI.test_torque_of_a_rotational_traction(bi_sphere())),
    ("particle stress on a sphere", PRB.test_particle_stress_on_a_sphere),
    ("probe pressure gauge", lambda: PRB.test_pressure_gauge_at_the_lower_wall(probe_field())),
    ("probe momentum balance", lambda: PRB.test_momentum_balance_away_from_sources(probe_field())),
]


# the pins that look at a module's own quantities run first for its mutants
# (every pin still runs until one fails)
FIRST = {
    "probes": ("probe pressure gauge", "probe momentum balance", "particle stress on a sphere"),
    "bi": ("element rule on polynomials", "vertex element in closed form",
           "double-layer vertex element with n~", "torque of a rotational traction"),
    "surface": ("surface velocity of a uniform density",),
    "fredholm": ("Fredholm operator on q = n",),
}


def first_failure(module=None):
    first = FIRST.get(module, ())
    order = [c for c in CHECKS if c[0] in first] + [c for c in CHECKS if c[0] not in first]
    for name, check in order:
        try:
            check()
        except AssertionError:
            return name
    return None


def test_control_passes_every_check():
    assert first_failure() is None


@pytest.mark.parametrize("mutation", sorted(MUTATIONS))
def test_mutation_is_caught(mutation, monkeypatch):
    install(monkeypatch, mutant(*MUTATIONS[mutation]))
    caught = first_failure(MUTATIONS[mutation][0])
    print(f"{mutation}: caught by {caught}")
    assert caught is not None, f"no pin fails for: {mutation}"
