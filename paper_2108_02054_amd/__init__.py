"""MI355X (gfx950) partial-reuse algebraic multigrid.

The hierarchy is built once (Algorithm 1 of Demidov, arXiv 2108.02054); on every later
time step the transfer operators are kept and the Galerkin operators, smoothers and the
coarsest solver are rebuilt (Algorithm 4), with the Galerkin products' patterns cached.
Solves use CG preconditioned by one V-cycle (Algorithm 2).  All of it runs in the HIP
library ``libamgmi.so``; this package only marshals arguments.
"""
from .amg import (  # noqa: F401
    AMG,
    AMGSolve,
    AmgError,
    AmgParams,
    EXPORTED,
    FULL,
    OPERATOR_ONLY,
    PARTIAL,
    default_params,
    lib,
    logcoef7_adjoint,
    logcoef7_assemble,
)
