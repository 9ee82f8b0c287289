"""FP64 CPU oracle of the GGEM slit evaluation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, double-precision
restatement of what the method computes, written from Kumar & Graham,
"Accelerated boundary integral method for multiphase flow in non-periodic
geometries" (GGEM split, Sec. 3.2; spectral slit solver, Appendix C).  It
shares no code with the HIP library.  Only the test suite, the smoke check
of ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it;
the product path never routes through it.
"""
from .ggem import (  # noqa: F401
    LOCAL, GLOBAL, ALL,
    SlitGrid,
    rho_g, stokeslet_local, pressure_local, stresslet_local,
    plane_primitive,
    local_velocity, local_traction, wall_data, spread, spread_at_nodes,
    dft_xz, idft_xz, cheb_forward_matrix, cheb_inverse_matrix,
    cheb_diff_matrix, helmholtz_tau, solve_modes, pressure_gauge,
    global_fields, interpolate, single_layer, double_layer,
)
from .fredholm import fredholm_apply, gauss_points, interpolate_to_gauss  # noqa: F401
from .surface import (  # noqa: F401
    node_normals, node_areas, laplace_beltrami_position, curvature, drop_rhs,
    surface_velocity,
)
from . import mlp  # noqa: F401
