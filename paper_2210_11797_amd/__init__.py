"""MI355X-native hybridised trace solver (HIP library + thin Python binding).

The compute path lives in libhyb.so (C ABI in include/hyb.h); this package only marshals
arguments to it.  Importing the package does not load the library; ``HybSolver`` does, and
raises if it has not been built.
"""

from ._native import (  # noqa: F401
    ABI_FUNCTIONS,
    GEOM_BOX,
    GEOM_SHELL,
    HYB_BREAKDOWN,
    HYB_DEBUG_NAN_STAGE,
    HYB_DEBUG_UNPAIRED_RESTRICT,
    HYB_DEBUG_ZERO_GAMMA,
    HYB_STAGNATED,
    HYB_NOT_CONVERGED,
    HYB_OK,
    LIB_PATH,
    PREC_FP64,
    PREC_MFMA_BF16X,
    PREC_MFMA_FP32,
    PREC_MIXED,
    HybSolver,
    Params,
    levels_of,
    solver_for,
    load,
)
