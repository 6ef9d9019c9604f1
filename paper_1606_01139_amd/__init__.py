"""MI355X-native partitioned shift-without-invert eigensolver and T(E).

The computation lives in the HIP library libtransec_gpu (csrc/, C-ABI in
include/transec_gpu.h); `binding` marshals arguments to it.
"""
from .binding import (Operator, TsgError, default_opts, dense_eig, load, solve_batch, FP64, FP32_BULK, PLAN_ALG1,
                      PLAN_EQUAL, PLAN_SAMPLED, PLAN_SEMICLASSICAL, SELECT_NEAREST, SELECT_SMALLEST_REAL, SELECT_LARGEST_REAL, EXPORTS,
                      TSG_OK, TSG_ENOCONV, TSG_EBREAKDOWN, EXTRACT_RITZ, EXTRACT_HARMONIC)

from .autograd import transmission as transmission_autograd

__all__ = ["transmission_autograd", "Operator", "TsgError", "default_opts", "dense_eig", "load", "solve_batch", "FP64", "FP32_BULK", "PLAN_ALG1",
           "PLAN_EQUAL", "PLAN_SAMPLED", "PLAN_SEMICLASSICAL", "SELECT_NEAREST", "SELECT_SMALLEST_REAL", "SELECT_LARGEST_REAL", "EXPORTS",
           "TSG_OK", "TSG_ENOCONV", "TSG_EBREAKDOWN", "EXTRACT_RITZ", "EXTRACT_HARMONIC"]
