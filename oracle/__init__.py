"""Python binding of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import
this package.  It shares no code with the HIP library.
"""
from .binding import (  # noqa: F401
    ORA_OK,
    OracleError,
    OracleHierarchy,
    OracleParams,
    aggregate,
    adjoint_logcoef7,
    assemble_logcoef7,
    build,
    lib,
    mix64,
    num_threads,
    set_num_threads,
)
