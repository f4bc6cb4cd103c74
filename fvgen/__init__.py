"""Seeded synthetic inputs for the unstructured finite-volume Euler step.

This package produces meshes, cell permutations, initial states and time
steps.  It holds no part of the step itself (no flux, no update): both the
CPU oracle and the HIP library consume what it builds, and neither imports
the other.
"""

from .mesh import Mesh, periodic_mesh, permute_mesh, SNAP_BITS
from .ic import (
    GAMMA,
    Primitive,
    vortex_primitive,
    vortex_exact_primitive,
    bumps_primitive,
    to_conserved,
    cfl_dt,
)

__all__ = [
    "Mesh",
    "periodic_mesh",
    "permute_mesh",
    "SNAP_BITS",
    "GAMMA",
    "Primitive",
    "vortex_primitive",
    "vortex_exact_primitive",
    "bumps_primitive",
    "to_conserved",
    "cfl_dt",
]
