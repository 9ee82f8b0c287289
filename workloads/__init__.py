"""Seeded synthetic workloads for the GGEM slit engine.

This package only draws geometry and random strengths.  It holds none of the
method's arithmetic, so both the CPU oracle and the GPU path may use it.
"""
from .inputs import (  # noqa: F401
    SlitCase,
    icosphere,
    case_small_sl,
    case_capsules_sl,
    case_capsules_dl,
    case_batched,
    random_case,
    node_normals,
    case_small_surface,
    DropCase,
    case_shear_drops,
    RigidSphereCase,
    case_rigid_sphere,
    CapsuleCase,
    case_capsule_suspension,
)
