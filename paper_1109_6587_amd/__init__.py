"""GGEM evaluation of Stokes flow in a planar slit on AMD MI355X (gfx950).

The computation lives in the HIP library ``libggem.so`` (C-ABI in
``include/ggem.h``); this package holds its sources (``csrc/``), the build
script and a ctypes binding with the same entry points.
"""
from .ggem import (  # noqa: F401
    FP64, MIXED, PART_ALL, PART_GLOBAL, PART_LOCAL, EXPORTS, GGEMError, Plan, load_library,
    FredholmSolver, Surface, MLP, MLP_PARAMS, Batch, single_layer_noalloc, RigidParticle,
    poiseuille, undisturbed_traction, FLOW_SHEAR, FLOW_POISEUILLE, INTERP_LAGRANGE, INTERP_SPECTRAL, Membrane,
)
