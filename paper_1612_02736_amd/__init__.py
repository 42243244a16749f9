"""MI355X-native HPS (Hierarchical Poincare-Steklov) direct solver.

The solver lives in the HIP/C++ library ``libhps.so`` (C ABI in
``include/hps.h``); ``hps`` is its ctypes binding and ``autograd`` wraps the
solve and its adjoint as a ``torch.autograd.Function``.
"""

from .hps import (HPS_BC_DIRICHLET, HPS_BC_NEUMANN, HPS_BC_PERIODIC, HPS_PREC_FP32,
                  HPS_PREC_FP64, HPS_PREC_MIXED, HPS_SOLVE_NOALLOC_MAX_BYTES, EXPORTS, HPSError, LIB_PATH, Solver, Tree,
                  lib)
from . import hps

__all__ = ["Tree", "Solver", "HPSError", "lib", "LIB_PATH", "EXPORTS",
           "HPS_PREC_FP64", "HPS_PREC_MIXED", "HPS_PREC_FP32", "HPS_SOLVE_NOALLOC_MAX_BYTES",
           "HPS_BC_DIRICHLET", "HPS_BC_NEUMANN", "HPS_BC_PERIODIC"]
