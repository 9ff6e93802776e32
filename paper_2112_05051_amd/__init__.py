"""MI355X-native solver for the 3-D Richards equation (arXiv 2112.05051).

The solver lives in librichards.so (HIP for gfx950, C-ABI in include/richards.h);
this package is its thin Python binding.  See `Solver` and `match_sweep`.
"""
from ._lib import (Solver, Server, RichError, match_sweep, query_bytes, load, status_string, stats_dict,
                   PREC_FP64, PREC_MIXED, WHICH_J, WHICH_A, WHICH_P, WHICH_PT, OK, STEP_TOO_SMALL, LIB_PATH, EXPORTS, KERNELS)

__all__ = ["Solver", "Server", "RichError", "match_sweep", "query_bytes", "load", "status_string", "stats_dict",
           "PREC_FP64", "PREC_MIXED", "WHICH_J", "WHICH_A", "WHICH_P", "WHICH_PT", "OK", "STEP_TOO_SMALL", "LIB_PATH", "EXPORTS", "KERNELS"]
