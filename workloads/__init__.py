"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This package holds input synthesis only (grid patterns, PDE coefficients, right-hand
sides, seeds).  None of the multigrid method's arithmetic lives here.
"""
from .poisson import (  # noqa: F401
    SEED_ROOT,
    STREAM_RHS,
    STREAM_UT,
    STREAM_THETA,
    STREAM_CELLS,
    STREAM_LOGN,
    STREAM_DRIFT,
    rng,
    stencil_pattern,
    pattern_7pt,
    pattern_27pt,
    two_fluid_7pt,
    front_c1,
    front_moving,
    lognormal_27pt,
    logcoef_inputs,
    logcoef_theta,
    rhs_uniform,
    neumann_7pt,
    CONFIGS,
    series_matrix,
)
