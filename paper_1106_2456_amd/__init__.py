"""MI355X multi-determinant evaluation by the table method (arXiv:1106.2456).

The computation lives in libmde.so (hand-written HIP for gfx950) behind the
C ABI of include/mde.h; this package is its thin Python binding.
"""
from ._lib import (MDE_FP64, MDE_MIXED, MDE_MIXED_GEMM, MDE_MIXED_GEMM_KSUM64, ST_NONFINITE, ST_SINGULAR_REF, ST_SMALL_RATIO,
                   ST_ZERO_PSI, LIB_PATH, MdeError, exported_symbols, lib)
from .context import Context, Graph, Group
from .autograd import MultiDetLogPsi

__all__ = ["Context", "Graph", "Group", "MultiDetLogPsi", "MdeError", "lib", "LIB_PATH",
           "exported_symbols", "MDE_FP64", "MDE_MIXED", "MDE_MIXED_GEMM", "MDE_MIXED_GEMM_KSUM64", "ST_SINGULAR_REF", "ST_SMALL_RATIO",
           "ST_NONFINITE", "ST_ZERO_PSI"]
