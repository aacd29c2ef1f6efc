"""MI355X (gfx950) FP64 implementation of the MSTAR regularised integrator.

The computation lives in libmstar.so (HIP kernels behind the C ABI of
include/mstar.h); this package only loads it and marshals arguments.
"""
from .mstar import (Context, MstarError, Params, Stats, BatchConfig, BATCH_STATS_DTYPE, lib, params, OK, W_TIME_TOL, E_INVAL, E_NOMEM,
                    E_DEVICE, E_NONFINITE, E_COINCIDENT, E_NOCONV, E_MAXSTEPS, E_UNSUPPORTED, DEVICE_PTRS, EAGER, MST_DC,
                    LIB_PATH, EXPORTS, force_noalloc, NOALLOC_MAX_N)

__all__ = ["Context", "MstarError", "Params", "Stats", "BatchConfig", "BATCH_STATS_DTYPE", "lib", "params",
           "LIB_PATH", "EXPORTS", "force_noalloc", "NOALLOC_MAX_N"]
