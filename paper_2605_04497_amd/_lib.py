"""ctypes declarations for libqtreeshap.so (the C-ABI in include/qtreeshap.h).

Argument marshalling only.  Importing this module loads the in-tree library and
raises if it has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtreeshap.so")

QTS_OK = 0
QTS_E_INVALID_ARG = -1
QTS_E_INVALID_MODEL = -2
QTS_E_UNSUPPORTED = -3
QTS_E_HIP = -4
QTS_E_OOM = -5
QTS_FP32 = 0
QTS_FP64 = 1

ERROR_NAMES = {QTS_E_INVALID_ARG: "QTS_E_INVALID_ARG", QTS_E_INVALID_MODEL: "QTS_E_INVALID_MODEL",
               QTS_E_UNSUPPORTED: "QTS_E_UNSUPPORTED", QTS_E_HIP: "QTS_E_HIP",
               QTS_E_OOM: "QTS_E_OOM"}

P = ctypes.c_void_p


class TreeArrays(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int32), ("tree_offsets", P), ("left", P), ("right", P),
                ("feature", P), ("threshold", P), ("default_left", P), ("cover", P),
                ("value", P)]


class Info(ctypes.Structure):
    _fields_ = [("n_features", ctypes.c_int32), ("n_trees", ctypes.c_int32),
                ("n_leaves", ctypes.c_int64), ("n_paths", ctypes.c_int64),
                ("n_elements", ctypes.c_int64), ("max_depth", ctypes.c_int32),
                ("max_unique", ctypes.c_int32), ("n_buckets", ctypes.c_int32),
                ("device", ctypes.c_int32), ("n_pair_classes", ctypes.c_int32),
                ("n_graphs", ctypes.c_int32), ("n_merged", ctypes.c_int64),
                ("n_value_paths", ctypes.c_int64), ("n_value_elements", ctypes.c_int64),
                ("n_pair_rows", ctypes.c_int64), ("n_pair_elements", ctypes.c_int64),
                ("n_pair_updates", ctypes.c_int64), ("n_value_shared", ctypes.c_int64),
                ("n_path_shared", ctypes.c_int64), ("n_value_segments", ctypes.c_int64),
                ("n_groups", ctypes.c_int32), ("pairs_dfs", ctypes.c_int32),
                ("n_dfs_nodes", ctypes.c_int64),
                ("n_dfs_updates", ctypes.c_int64), ("n_dfs_updates3", ctypes.c_int64),
                ("n_value_prefix_kept", ctypes.c_int64), ("n_path_prefix_kept", ctypes.c_int64)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "qts_load_ensemble": (ctypes.c_int, [ctypes.POINTER(TreeArrays), ctypes.c_int32,
                                         ctypes.c_double, P, ctypes.POINTER(P)]),
    "qts_build_host": (ctypes.c_int, [ctypes.POINTER(TreeArrays), ctypes.c_int32,
                                      ctypes.c_double, ctypes.POINTER(P)]),
    "qts_load_ensemble_grouped": (ctypes.c_int, [ctypes.POINTER(TreeArrays), P, ctypes.c_int32,
                                                 ctypes.c_int32, P, P, ctypes.POINTER(P)]),
    "qts_build_host_grouped": (ctypes.c_int, [ctypes.POINTER(TreeArrays), P, ctypes.c_int32,
                                              ctypes.c_int32, P, ctypes.POINTER(P)]),
    "qts_free_ensemble": (ctypes.c_int, [P]),
    "qts_expected_values": (ctypes.c_int, [P, P]),
    "qts_expected_value": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double)]),
    "qts_num_leaves": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int64)]),
    "qts_get_info": (ctypes.c_int, [P, ctypes.POINTER(Info)]),
    "qts_export_paths": (ctypes.c_int, [P] + [P] * 9),
    "qts_gauss_legendre": (ctypes.c_int, [ctypes.c_int32, P, P, P]),
    "qts_shap_values": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_int64, P, P,
                                       ctypes.c_int, P]),
    "qts_shap_values_noalloc": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_int64, P, P,
                                               ctypes.c_int, P]),
    "qts_shap_interactions": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_int64, P, P, P,
                                             ctypes.c_int, P]),
    "qts_shap_interactions3": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_int64, P, P,
                                              ctypes.c_int, P]),
    "qts_shap_backward": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_int64, P, P,
                                         ctypes.c_int, P]),
    "qts_autotune": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_int, P]),
    "qts_get_launch_shape": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "qts_set_graph_replay": (ctypes.c_int, [P, ctypes.c_int32]),
    "qts_set_sibling_merge": (ctypes.c_int, [P, ctypes.c_int32]),
    "qts_set_node_policy": (ctypes.c_int, [P, ctypes.c_int32]),
    "qts_set_deterministic": (ctypes.c_int, [P, ctypes.c_int32]),
    "qts_debug_fail_allocations": (ctypes.c_int, [ctypes.c_int64]),
    "qts_set_pair_traversal": (ctypes.c_int, [P, ctypes.c_int32]),
    "qts_set_tune_cache": (ctypes.c_int, [ctypes.c_char_p]),
    "qts_tune_cache_stats": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "qts_set_kernel_timing": (ctypes.c_int, [ctypes.c_int32]),
    "qts_kernel_timing_read": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "qts_last_error": (ctypes.c_char_p, []),
}


class QtsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "QTS_ERROR"), code, msg))
        self.code = code


_lib = None


def lib():
    """Load the in-tree library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libqtreeshap.so is not built (%s); build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != QTS_OK:
        raise QtsError(rc, lib().qts_last_error().decode("utf-8", "replace"))
