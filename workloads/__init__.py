"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates problem data* (grid points, coefficient fields,
the finite element stiffness matrix of the model problem, the boundary element
matrix of the second model problem with the low-rank factors of its far-field
blocks, Gaussian factors and right-hand sides).  It contains none of the arithmetic of the H^2 method
itself, so both the CPU oracle and the HIP path can consume the same inputs
without sharing any implementation.
"""

from .fem import (  # noqa: F401
    grid_points,
    sigma_subdomains_2d,
    sigma_blocks_3d,
    fem2d_p1,
    fem3d_q1,
    convection_x,
    gaussian,
    problem,
)
from . import bem  # noqa: F401,E402
