"""Seeded synthetic inputs shared by the CPU oracle and the HIP library.

This package only *describes* a workload: mesh geometry, material and slot
maps, source and time-grid constants, solver settings and seeded random
arrays.  It holds none of the method's arithmetic (no assembly, no PWM
evaluation, no time stepping, no grid transfers); each consumer computes those
on its own.
"""

from .machine import (  # noqa: F401
    R_IN, R_OUT, MU0, MATERIALS, MAT_ROTOR_IRON, MAT_BAR, MAT_AIR, MAT_SLOT,
    MAT_STATOR_IRON, N_BARS, PolarMesh, polar_mesh, Source, BHLaw, Circuit,
)
from .configs import Config, LevelSpec, config, CONFIG_NAMES, hierarchy  # noqa: F401
