"""Seeded synthetic inputs shared by the oracle-based tests and the GPU path.

This package holds meshes (vertex coordinates, element-to-vertex lists, face
tags), closed-form initial fields in macroscopic variables (density, velocity),
time-step and parameter choices for the workloads the paper runs.  It holds
none of the method's arithmetic: converting macroscopic fields into moments,
operators, fluxes and the time integrator live on each side separately.
"""
from .meshes import kuhn_cube, ogrid_airfoil, periodic_square  # noqa: F401
from .fields import taylor_green_2d, taylor_green_3d  # noqa: F401
from .configs import CASES, cfl_dt, make_case  # noqa: F401
