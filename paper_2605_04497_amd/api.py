"""Python binding of the qtreeshap C-ABI: ensembles, Shapley values, pairwise
interactions and the leaf-value adjoint on MI355X.

Argument marshalling only: every computation runs in the HIP library.  PyTorch
supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp32": L.QTS_FP32, "fp64": L.QTS_FP64}
_DTYPE = {"fp32": torch.float32, "fp64": torch.float64}


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def gauss_legendre(n: int = 8):
    """(t, 1-t, w): the n-node Gauss-Legendre rule on [0,1] built by the library."""
    t, s, w = np.zeros(n), np.zeros(n), np.zeros(n)
    L.check(L.lib().qts_gauss_legendre(n, t.ctypes.data, s.ctypes.data, w.ctypes.data))
    return t, s, w


def set_tune_cache(path) -> None:
    """Keep autotuned launch shapes in the text file `path` (None: off)."""
    L.check(L.lib().qts_set_tune_cache(None if path is None else str(path).encode()))


def tune_cache_stats():
    """(hits, misses) of the autotune cache since it was set."""
    h, m = ctypes.c_int64(), ctypes.c_int64()
    L.check(L.lib().qts_tune_cache_stats(ctypes.byref(h), ctypes.byref(m)))
    return int(h.value), int(m.value)


KERNEL_KINDS = {"interactions3": 3, "values": 0, "interactions": 1, "backward": 2}


def set_kernel_timing(enable: bool) -> None:
    """Record HIP events around the main kernel launches of each call."""
    L.check(L.lib().qts_set_kernel_timing(1 if enable else 0))


def read_kernel_timing(kind: str = "values"):
    """(total_ms, calls) of the main kernel of `kind` since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    L.check(L.lib().qts_kernel_timing_read(KERNEL_KINDS[kind], ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, int(n.value)


class Ensemble:
    """A tree ensemble loaded into the library.

    `model` is any object with the structure-of-arrays fields tree_offsets,
    left, right, feature, threshold, default_left, cover, value, n_features
    (and optionally base_score); see include/qtreeshap.h for their meaning.
    With host_only=True the path table is built but no device is touched.
    """

    def __init__(self, model, host_only: bool = False, device=None):
        a = {k: np.ascontiguousarray(getattr(model, k), dt) for k, dt in (
            ("tree_offsets", np.int64), ("left", np.int32), ("right", np.int32),
            ("feature", np.int32), ("threshold", np.float32), ("default_left", np.uint8),
            ("cover", np.float64), ("value", np.float64))}
        self.n_features = int(model.n_features)
        n_trees = int(a["tree_offsets"].shape[0] - 1)
        # multi-output models: tree_group [T] and n_groups (base_score then
        # holds one value per group)
        tg = getattr(model, "tree_group", None)
        self.n_groups = int(getattr(model, "n_groups", 1) or 1) if tg is not None else 1
        bs = np.ascontiguousarray(np.broadcast_to(
            np.asarray(getattr(model, "base_score", 0.0), np.float64).reshape(-1),
            (self.n_groups,)))
        tg = np.ascontiguousarray(tg if tg is not None else np.zeros(n_trees), np.int32)
        ta = L.TreeArrays(n_trees,
                          *[a[k].ctypes.data for k in ("tree_offsets", "left", "right", "feature",
                                                       "threshold", "default_left", "cover",
                                                       "value")])
        h = ctypes.c_void_p()
        if host_only:
            self.device = None
            L.check(L.lib().qts_build_host_grouped(ctypes.byref(ta), tg.ctypes.data,
                                                   self.n_groups, self.n_features,
                                                   bs.ctypes.data, ctypes.byref(h)))
        else:
            self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
                else torch.device(device)
            with torch.cuda.device(self.device):
                L.check(L.lib().qts_load_ensemble_grouped(
                    ctypes.byref(ta), tg.ctypes.data, self.n_groups, self.n_features,
                    bs.ctypes.data, _stream_ptr(self.device), ctypes.byref(h)))
        self._h = h
        info = L.Info()
        L.check(L.lib().qts_get_info(self._h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in L.Info._fields_}
        ev = np.zeros(self.n_groups)
        L.check(L.lib().qts_expected_values(self._h, ev.ctypes.data))
        # one output: a float; several: one value per output group
        self.expected_value = float(ev[0]) if self.n_groups == 1 else ev
        self.n_leaves = int(info.n_leaves)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            if self.device is not None:
                torch.cuda.synchronize(self.device)
            L.check(L.lib().qts_free_ensemble(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- checks
    def _rows(self, X: torch.Tensor):
        if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
            raise TypeError("X must be a CUDA/HIP float32 tensor")
        if X.dtype != torch.float32 or X.dim() != 2:
            raise TypeError("X must be a 2-D float32 tensor")
        if X.shape[1] < self.n_features:
            raise ValueError("X has %d columns, the model needs %d" % (X.shape[1],
                                                                        self.n_features))
        if X.stride(1) != 1:
            X = X.contiguous()
        return X, X.shape[0], X.stride(0)

    @staticmethod
    def _out(t, shape, dtype, device, what):
        """Check a caller-supplied output buffer before any library call: the
        kernels write through its raw device pointer, so a wrong size, type,
        layout or device must be rejected here."""
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % what)
        if t.device != device:
            raise ValueError("%s is on %s, X is on %s" % (what, t.device, device))
        if t.dtype != dtype:
            raise TypeError("%s must be %s for this precision, got %s" % (what, dtype, t.dtype))
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (what, tuple(shape),
                                                                tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % what)
        return t

    def _leaf(self, leaf_values, device):
        if leaf_values is None:
            return None
        if (not isinstance(leaf_values, torch.Tensor) or leaf_values.dtype != torch.float64
                or leaf_values.device != device or leaf_values.numel() != self.n_leaves):
            raise TypeError("leaf_values must be a float64 tensor of n_leaves values on the "
                            "device of X")
        return leaf_values.contiguous()

    # ---------------------------------------------------------------- compute
    def _per_sample(self, M, *rest):
        """Output shape: [M, *rest], or [M, n_groups, *rest] for several outputs."""
        return (M,) + ((self.n_groups,) if self.n_groups > 1 else ()) + tuple(rest)

    def shap_values(self, X: torch.Tensor, precision: str = "fp32", leaf_values=None,
                    out=None) -> torch.Tensor:
        """phi[M, F] ([M, n_groups, F] for a multi-output model); float32 for
        'fp32', float64 for 'fp64'."""
        X, M, ldx = self._rows(X)
        lv = self._leaf(leaf_values, X.device)
        shape = self._per_sample(M, self.n_features)
        if out is None:
            out = torch.empty(shape, dtype=_DTYPE[precision], device=X.device)
        else:
            self._out(out, shape, _DTYPE[precision], X.device, "out")
        L.check(L.lib().qts_shap_values(self._h, _ptr(X), M, ldx, _ptr(lv), _ptr(out),
                                        _PREC[precision], _stream_ptr(X.device)))
        return out

    def shap_interactions(self, X: torch.Tensor, precision: str = "fp32", leaf_values=None,
                          with_phi: bool = False, out=None, out_phi=None):
        """Phi[M, F, F] (and phi[M, F] when with_phi); with several outputs
        [M, n_groups, F, F] and [M, n_groups, F]."""
        X, M, ldx = self._rows(X)
        lv = self._leaf(leaf_values, X.device)
        F = self.n_features
        dt = _DTYPE[precision]
        if out is not None:
            Phi = self._out(out, self._per_sample(M, F, F), dt, X.device, "out")
        else:
            Phi = torch.empty(self._per_sample(M, F, F), dtype=dt, device=X.device)
        phi = None
        if with_phi:
            if out_phi is not None:
                phi = self._out(out_phi, self._per_sample(M, F), dt, X.device, "out_phi")
            else:
                phi = torch.empty(self._per_sample(M, F), dtype=dt, device=X.device)
        elif out_phi is not None:
            raise ValueError("out_phi is given but with_phi is False")
        L.check(L.lib().qts_shap_interactions(self._h, _ptr(X), M, ldx, _ptr(lv), _ptr(phi),
                                              _ptr(Phi), _PREC[precision],
                                              _stream_ptr(X.device)))
        return (Phi, phi) if with_phi else Phi

    def shap_interactions3(self, X: torch.Tensor, precision: str = "fp32",
                           leaf_values: torch.Tensor | None = None, out=None) -> torch.Tensor:
        """Third-order Shapley interaction indices, packed [M, F(F-1)(F-2)/6]
        ([M, n_groups, ...] with several outputs): the triple of features
        i < j < k at k(k-1)(k-2)/6 + j(j-1)/2 + i."""
        X, M, ldx = self._rows(X)
        F = self.n_features
        T3 = F * (F - 1) * (F - 2) // 6
        dt = _DTYPE[precision]
        if out is None:
            out = torch.empty(self._per_sample(M, T3), dtype=dt, device=X.device)
        else:
            self._out(out, self._per_sample(M, T3), dt, X.device, "out")
        lv = self._leaf(leaf_values, X.device)
        L.check(L.lib().qts_shap_interactions3(self._h, _ptr(X), M, ldx, _ptr(lv), _ptr(out),
                                               _PREC[precision], _stream_ptr(X.device)))
        return out

    @staticmethod
    def triples_dense(packed: torch.Tensor, n_features: int) -> torch.Tensor:
        """Expand a packed [..., F(F-1)(F-2)/6] tensor to the symmetric
        [..., F, F, F] one (zero where two indices coincide)."""
        F = n_features
        lead = tuple(packed.shape[:-1])
        packed = packed.reshape(-1, packed.shape[-1])
        idx = torch.combinations(torch.arange(F, device=packed.device), 3)  # i < j < k
        i, j, k = idx[:, 0], idx[:, 1], idx[:, 2]
        pos = k * (k - 1) * (k - 2) // 6 + j * (j - 1) // 2 + i
        dense = torch.zeros((packed.shape[0], F, F, F), dtype=packed.dtype, device=packed.device)
        v = packed[:, pos]
        for a, b, c in ((i, j, k), (i, k, j), (j, i, k), (j, k, i), (k, i, j), (k, j, i)):
            dense[:, a, b, c] = v
        return dense.reshape(lead + (F, F, F))

    def shap_backward(self, X: torch.Tensor, grad_phi: torch.Tensor,
                      precision: str = "fp32", out=None) -> torch.Tensor:
        """grad_leaf[n_leaves] (float64) = J^T grad_phi."""
        X, M, ldx = self._rows(X)
        if not isinstance(grad_phi, torch.Tensor):
            raise TypeError("grad_phi must be a torch tensor")
        if grad_phi.device != X.device:
            raise ValueError("grad_phi is on %s, X is on %s" % (grad_phi.device, X.device))
        if tuple(grad_phi.shape) != self._per_sample(M, self.n_features):
            raise ValueError("grad_phi must be [M, F] ([M, n_groups, F] with several outputs)")
        g = grad_phi.to(_DTYPE[precision]).contiguous()
        if out is None:
            out = torch.empty(self.n_leaves, dtype=torch.float64, device=X.device)
        else:
            self._out(out, (self.n_leaves,), torch.float64, X.device, "out")
        L.check(L.lib().qts_shap_backward(self._h, _ptr(X), M, ldx, _ptr(g), _ptr(out),
                                          _PREC[precision], _stream_ptr(X.device)))
        return out

    def autotune(self, M_hint: int, precision: str = "fp32"):
        """Time candidate launch shapes on M_hint synthetic rows; keep the fastest."""
        L.check(L.lib().qts_autotune(self._h, int(M_hint), _PREC[precision],
                                     _stream_ptr(self.device)))

    def launch_shape(self, kind: str, precision: str = "fp32", index: int = 0):
        """(waves per workgroup, target work items) of first-order bucket `index`
        (kind 'values') or adjoint bucket `index` (kind 'adjoint'), or (largest
        path chunk, least work items) of interactions class `index` (kind
        'interactions')."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().qts_get_launch_shape(self._h, {"values": 0, "interactions": 1, "adjoint": 2}[kind],
                                             _PREC[precision], int(index), ctypes.byref(a),
                                             ctypes.byref(b)))
        return a.value, b.value

    def set_graph_replay(self, enable: bool = True):
        """Capture each call once into a HIP graph and replay it on later calls
        with the same tensors (pass `out=` to reuse output buffers)."""
        with torch.cuda.device(self.device):
            L.check(L.lib().qts_set_graph_replay(self._h, int(bool(enable))))

    def set_sibling_merge(self, enable: bool = True):
        """First-order calls walk one merged path per pair of sibling leaves
        (default) or every path (exact same values up to rounding)."""
        L.check(L.lib().qts_set_sibling_merge(self._h, int(bool(enable))))

    def set_pair_traversal(self, traversal: str = "auto"):
        """'paths': the interactions call walks collapsed paths; 'dfs':
        Algorithm 1's depth-first form (one pair update per internal node and
        feature split above it); 'auto' (default): the faster of the two, as
        found by the next autotune of each precision (paths until then)."""
        with torch.cuda.device(self.device):
            L.check(L.lib().qts_set_pair_traversal(
                self._h, {"paths": 0, "dfs": 1, "auto": 2}[traversal]))
        self.refresh_info()

    def set_deterministic(self, enable: bool = True):
        """First-order values and the adjoint identical bit for bit from run to
        run (ordered sums without atomics; the values call runs slower)."""
        L.check(L.lib().qts_set_deterministic(self._h, int(bool(enable))))

    def set_node_policy(self, policy: str = "fixed8"):
        """'fixed8': the 8-node rule everywhere (default); 'exact': the fewest
        nodes exact by Theorem 2 where that is fewer than 8 (first order and
        adjoint: 4 for paths of at most 8 features; interactions: 2, 4, 6 for
        capacity classes 4, 8, 12)."""
        L.check(L.lib().qts_set_node_policy(self._h, {"fixed8": 0, "exact": 1}[policy]))

    def refresh_info(self) -> dict:
        info = L.Info()
        L.check(L.lib().qts_get_info(self._h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in L.Info._fields_}
        return self.info

    # ---------------------------------------------------------------- inspection
    def export_paths(self) -> dict:
        """The collapsed path table (host copies)."""
        n_p, n_e = self.info["n_paths"], self.info["n_elements"]
        out = {"path_leaf": np.zeros(n_p, np.int32), "path_len": np.zeros(n_p, np.int32),
               "path_off": np.zeros(n_p, np.int32), "feat": np.zeros(n_e, np.int32),
               "lo": np.zeros(n_e, np.float32), "hi": np.zeros(n_e, np.float32),
               "missing_ok": np.zeros(n_e, np.uint8), "b": np.zeros(n_e),
               "one_minus_b": np.zeros(n_e)}
        L.check(L.lib().qts_export_paths(self._h, *[out[k].ctypes.data for k in (
            "path_leaf", "path_len", "path_off", "feat", "lo", "hi", "missing_ok", "b",
            "one_minus_b")]))
        return out


class ShapValues(torch.autograd.Function):
    """phi = ShapValues.apply(leaf_values, X, ensemble, precision).

    phi is linear in the leaf values; backward calls the library's adjoint.
    It is piecewise constant in X, so X receives no gradient."""

    @staticmethod
    def forward(ctx, leaf_values, X, ensemble, precision="fp32"):
        ctx.ensemble = ensemble
        ctx.precision = precision
        ctx.save_for_backward(X)
        return ensemble.shap_values(X, precision, leaf_values=leaf_values.detach())

    @staticmethod
    def backward(ctx, grad_phi):
        (X,) = ctx.saved_tensors
        g = ctx.ensemble.shap_backward(X, grad_phi, ctx.precision)
        return g, None, None, None
