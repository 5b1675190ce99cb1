"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package draws random numbers and builds coefficient fields and
right-hand sides.  It holds none of the factorization's arithmetic: no
matrix assembly, no elimination, no interpolative decomposition.
"""
from .workloads import (  # noqa: F401
    WORKLOADS,
    Workload,
    coeff_shape,
    make_coefficients,
    make_rhs,
    workload,
)
