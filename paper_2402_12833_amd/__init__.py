"""amgmpcg: additive-multigrid MPCG on AMD MI355X (HIP, gfx950).

The solver lives in ``libamgmpcg.so`` (HIP kernels + C ABI, header
``include/amgmpcg.h``); ``binding`` marshals arguments to it with ctypes.
"""
from .binding import (  # noqa: F401
    AmgMpcgError, BatchedSolver, Network, Solver, cnn_weight_count, CNN_LAYERS, default_options, gram_pinv, gram_pinv_noalloc, header_functions, last_error, load, status_string,
    OK, MAXIT, BREAKDOWN, INVALID_ARG, NOT_SPD, DIM_MISMATCH, NONFINITE, OOM, HIP_ERROR, UNAVAILABLE,
    MPCG, ADDITIVE_PCG, VCYCLE_PCG,
)
