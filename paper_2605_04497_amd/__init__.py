"""Quadrature-TreeSHAP on AMD Instinct MI355X (gfx950).

Path-Dependent TreeSHAP values, pairwise Shapley interactions and the adjoint
to leaf values, computed by hand-written HIP kernels behind the C-ABI in
include/qtreeshap.h.  Importing the package loads the in-tree library and
fails if it has not been built.
"""
from ._lib import QtsError, lib
from .api import (Ensemble, ShapValues, gauss_legendre, read_kernel_timing, set_kernel_timing,
                  set_tune_cache, tune_cache_stats)

lib()

__all__ = ["Ensemble", "ShapValues", "gauss_legendre", "QtsError", "lib", "set_kernel_timing",
           "read_kernel_timing", "set_tune_cache", "tune_cache_stats"]
