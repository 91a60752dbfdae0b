"""MI355X (gfx950) evaluator of cDFT excess chemical potentials.

The hot path is hand-written HIP behind the C ABI in include/pnp_cdft.h;
this package only marshals arguments to it (see ``binding``).  Importing it
does not load the library; the first call does, and fails loudly when the
library has not been built.
"""
from .binding import (PASS_NAMES, PnpError, Evaluator, Pool, Plan, bulk_mu_ex, lib_path, load_library, STATUS_NAMES,
                      TERM_HS, TERM_EC, TERM_SW, TERM_ALL, TERM_HS_WB, FP64, MIXED, FLAG_ASYNC, FLAG_APERIODIC, FLAG_CUBIC)

__all__ = ["PASS_NAMES", "PnpError", "Evaluator", "Pool", "Plan", "bulk_mu_ex", "lib_path", "load_library", "STATUS_NAMES",
           "TERM_HS", "TERM_EC", "TERM_SW", "TERM_ALL", "TERM_HS_WB", "FP64", "MIXED", "FLAG_ASYNC", "FLAG_APERIODIC", "FLAG_CUBIC"]
