"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package defines *problem data* only (grids, coefficient fields, right-hand
sides).  It holds none of the projection method's arithmetic, so both sides of
a parity test can draw identical inputs from it without sharing numerics.
"""
from .problems import (  # noqa: F401
    Operator,
    laplace2d,
    fv3d,
    fd2d_variable,
    fd1d_dense,
    fe_p1_2d,
    gaussian_C,
    uniform_C,
    batch_c5,
    random_band_T,
)
