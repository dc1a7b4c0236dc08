"""Error measures shared by the GPU parity tests.

Tolerances: the FP32 path must reach a row-normwise relative error of 1e-5
against the FP64 oracle, the FP64 path 1e-10:
    rel = max over rows r of  max_i |gpu[r,i] - oracle[r,i]| / max_i |oracle[r,i]|
(for Phi the row is one sample's F x F matrix).  A per-element relative
criterion is not reachable even by exact FP32 arithmetic: entries far below a
row's largest value carry the absolute rounding of that row's sums.
"""
import numpy as np

TOL_FP32 = 1e-5
TOL_FP64 = 1e-10


def row_normwise(got, want, floor=1e-30):
    got = np.asarray(got, np.float64).reshape(got.shape[0], -1)
    want = np.asarray(want, np.float64).reshape(want.shape[0], -1)
    if got.shape[0] == 0:
        return 0.0
    err = np.abs(got - want).max(axis=1)
    scale = np.maximum(np.abs(want).max(axis=1), floor)
    return float((err / scale).max())


def check(got, want, precision, what=""):
    tol = TOL_FP32 if precision == "fp32" else TOL_FP64
    rel = row_normwise(got, want)
    assert rel <= tol, "%s %s row-normwise rel err %.3e > %.0e" % (what, precision, rel, tol)
    return rel
