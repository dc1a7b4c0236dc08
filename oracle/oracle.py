"""Driver for the FP64 CPU oracle (qts_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports or links
anything here, and nothing here imports the GPU library.

Output conventions (readings of the paper, listed with the tests):
  phi[M,F]    Shapley values of the path-dependent game (Eq. 3, Eq. 9 with |S|=1)
  sii[M,F,F]  Shapley interaction index of each ordered pair i != k (Eq. 9, |S|=2)
  Phi[M,F,F]  interaction matrix: Phi[i,k] = SII_ik / 2 for i != k and
              Phi[i,i] = phi_i - sum_{k != i} Phi[i,k], so each row sums to phi
  expected    E[f] = v(empty set) summed over trees, plus the base score
Multi-output models (a group per tree) are computed per group on the group's
sub-ensemble; the *_grouped functions stack the results as [M, K, ...].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qts_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

N_METHOD = 8     # the fixed node count of the method (section 5)
N_EXACT = 32     # exact for d <= 64 at first order (Theorem 2)


def build() -> str:
    """Compile the oracle with gcc (plain C, -O2, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-shared", "-fPIC",
                           "-pthread", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        for name in ("orc_gauss_legendre", "orc_shap_values", "orc_shap_interactions",
                     "orc_leaf_grad", "orc_expected_value", "orc_predict", "orc_treeshap"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def default_threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


class _Model(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int32), ("tree_offsets", ctypes.c_void_p),
                ("left", ctypes.c_void_p), ("right", ctypes.c_void_p),
                ("feature", ctypes.c_void_p), ("threshold", ctypes.c_void_p),
                ("default_left", ctypes.c_void_p), ("cover", ctypes.c_void_p),
                ("value", ctypes.c_void_p), ("n_features", ctypes.c_int32)]


class OracleModel:
    """Holds contiguous copies of the ensemble arrays for the C oracle."""

    def __init__(self, ens):
        self.ens = ens
        self._keep = [np.ascontiguousarray(ens.tree_offsets, np.int64),
                      np.ascontiguousarray(ens.left, np.int32),
                      np.ascontiguousarray(ens.right, np.int32),
                      np.ascontiguousarray(ens.feature, np.int32),
                      np.ascontiguousarray(ens.threshold, np.float32),
                      np.ascontiguousarray(ens.default_left, np.uint8),
                      np.ascontiguousarray(ens.cover, np.float64),
                      np.ascontiguousarray(ens.value, np.float64)]
        self.F = int(ens.n_features)
        self.base_score = float(ens.base_score)
        self.n_leaves = int((self._keep[1] < 0).sum())
        self.struct = _Model(int(ens.n_trees), *[a.ctypes.data for a in self._keep], self.F)

    def ref(self):
        return ctypes.byref(self.struct)


def _model(m) -> OracleModel:
    return m if isinstance(m, OracleModel) else OracleModel(m)


def _X(X):
    X = np.ascontiguousarray(X, np.float32)
    return X, X.shape[0], X.shape[1]


def gauss_legendre(n: int):
    """(t, s=1-t, omega) of the n-point rule on [0,1], in FP64."""
    t = np.zeros(n); s = np.zeros(n); w = np.zeros(n)
    P = ctypes.c_void_p
    rc = lib().orc_gauss_legendre(ctypes.c_int(n), P(t.ctypes.data), P(s.ctypes.data),
                                  P(w.ctypes.data))
    if rc != 0:
        raise ValueError("bad node count %d" % n)
    return t, s, w


def shap_values(m, X, n=N_METHOD, threads=None) -> np.ndarray:
    m = _model(m)
    X, M, ld = _X(X)
    phi = np.zeros((M, m.F))
    rc = lib().orc_shap_values(m.ref(), ctypes.c_void_p(X.ctypes.data), ctypes.c_int64(M),
                               ctypes.c_int64(ld), ctypes.c_int(n),
                               ctypes.c_void_p(phi.ctypes.data),
                               ctypes.c_int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("orc_shap_values failed")
    return phi


def shap_sii(m, X, n=N_METHOD, threads=None):
    """(phi[M,F], sii[M,F,F]) with sii the raw pair indices (diagonal 0)."""
    m = _model(m)
    X, M, ld = _X(X)
    phi = np.zeros((M, m.F))
    sii = np.zeros((M, m.F, m.F))
    rc = lib().orc_shap_interactions(m.ref(), ctypes.c_void_p(X.ctypes.data),
                                     ctypes.c_int64(M), ctypes.c_int64(ld), ctypes.c_int(n),
                                     ctypes.c_void_p(phi.ctypes.data),
                                     ctypes.c_void_p(sii.ctypes.data),
                                     ctypes.c_int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("orc_shap_interactions failed")
    return phi, sii


def interaction_matrix(phi, sii) -> np.ndarray:
    """Phi with off-diagonal SII/2 and the diagonal that makes rows sum to phi."""
    Phi = 0.5 * sii.copy()
    idx = np.arange(phi.shape[1])
    Phi[:, idx, idx] = 0.0
    Phi[:, idx, idx] = phi - Phi.sum(axis=2)
    return Phi


def shap_interactions(m, X, n=N_METHOD, threads=None):
    phi, sii = shap_sii(m, X, n, threads)
    return phi, interaction_matrix(phi, sii)


def shap_sii3(m, X, n=N_METHOD, threads=None) -> np.ndarray:
    """sii3[M,F,F,F]: third-order Shapley interaction indices (Theorem 1 with
    |S| = 3, Eq. 9-10) of every ordered triple of distinct features; entries
    with a repeated index are 0."""
    m = _model(m)
    X, M, ld = _X(X)
    sii3 = np.zeros((M, m.F, m.F, m.F))
    rc = lib().orc_shap_sii3(m.ref(), ctypes.c_void_p(X.ctypes.data), ctypes.c_int64(M),
                             ctypes.c_int64(ld), ctypes.c_int(n),
                             ctypes.c_void_p(sii3.ctypes.data),
                             ctypes.c_int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("orc_shap_sii3 failed")
    return sii3


def leaf_grad(m, X, G, n=N_METHOD, threads=None) -> np.ndarray:
    """grad_leaf = J^T G with J[s,i,leaf] = d phi[s,i] / d val(leaf); leaves in
    tree-major node-id order."""
    m = _model(m)
    X, M, ld = _X(X)
    G = np.ascontiguousarray(G, np.float64)
    assert G.shape == (M, m.F)
    out = np.zeros(m.n_leaves)
    rc = lib().orc_leaf_grad(m.ref(), ctypes.c_void_p(X.ctypes.data), ctypes.c_int64(M),
                             ctypes.c_int64(ld), ctypes.c_int(n),
                             ctypes.c_void_p(G.ctypes.data), ctypes.c_void_p(out.ctypes.data),
                             ctypes.c_int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("orc_leaf_grad failed")
    return out


def expected_value(m) -> float:
    m = _model(m)
    out = ctypes.c_double(0.0)
    if lib().orc_expected_value(m.ref(), ctypes.byref(out)) != 0:
        raise RuntimeError("orc_expected_value failed")
    return out.value + m.base_score


def predict(m, X) -> np.ndarray:
    m = _model(m)
    X, M, ld = _X(X)
    out = np.zeros(M)
    if lib().orc_predict(m.ref(), ctypes.c_void_p(X.ctypes.data), ctypes.c_int64(M),
                         ctypes.c_int64(ld), ctypes.c_void_p(out.ctypes.data)) != 0:
        raise RuntimeError("orc_predict failed")
    return out + m.base_score


def treeshap(m, X, threads=None) -> np.ndarray:
    """phi by recursive TreeSHAP (an independent exact route; needs non-zero covers)."""
    m = _model(m)
    X, M, ld = _X(X)
    phi = np.zeros((M, m.F))
    if lib().orc_treeshap(m.ref(), ctypes.c_void_p(X.ctypes.data), ctypes.c_int64(M),
                          ctypes.c_int64(ld), ctypes.c_void_p(phi.ctypes.data),
                          ctypes.c_int(threads or default_threads())) != 0:
        raise RuntimeError("orc_treeshap failed")
    return phi


# ---------------------------------------------------------------------------
# Multi-output ensembles.  Each tree adds to the output of its group, so the
# game of output g is the sum of the path-dependent games (Eq. 3) of group g's
# trees, and every quantity above is computed per group on that group's
# sub-ensemble: a plain composition of the single-output oracle.
# ---------------------------------------------------------------------------

def _groups(ens):
    K = int(getattr(ens, "n_groups", 1) or 1)
    return K, [ens.group_trees(g) if K > 1 else list(range(ens.n_trees)) for g in range(K)]


def _base(ens, g):
    b = np.asarray(ens.base_score, np.float64).reshape(-1)
    return float(b[g] if b.shape[0] > 1 else b[0])


def _sub(ens, trees):
    sub = ens.subset_trees(trees)
    sub.base_score = 0.0
    return sub


def shap_values_grouped(ens, X, n=N_METHOD, threads=None) -> np.ndarray:
    """phi[M, K, F]: Shapley values of each output's game."""
    K, tg = _groups(ens)
    return np.stack([shap_values(_sub(ens, t), X, n, threads) for t in tg], axis=1)


def shap_interactions_grouped(ens, X, n=N_METHOD, threads=None):
    """(phi[M, K, F], Phi[M, K, F, F]) of each output's game."""
    K, tg = _groups(ens)
    parts = [shap_interactions(_sub(ens, t), X, n, threads) for t in tg]
    return (np.stack([p[0] for p in parts], axis=1), np.stack([p[1] for p in parts], axis=1))


def shap_sii3_grouped(ens, X, n=N_METHOD, threads=None) -> np.ndarray:
    """sii3[M, K, F, F, F] of each output's game."""
    K, tg = _groups(ens)
    return np.stack([shap_sii3(_sub(ens, t), X, n, threads) for t in tg], axis=1)


def expected_values_grouped(ens) -> np.ndarray:
    """E_g[f] + base score of each output."""
    K, tg = _groups(ens)
    return np.array([expected_value(_sub(ens, t)) + _base(ens, g) for g, t in enumerate(tg)])


def predict_grouped(ens, X) -> np.ndarray:
    """f_g(x) + base score of each output: [M, K]."""
    K, tg = _groups(ens)
    return np.stack([predict(_sub(ens, t), X) + _base(ens, g) for g, t in enumerate(tg)], axis=1)


def leaf_grad_grouped(ens, X, G, n=N_METHOD, threads=None) -> np.ndarray:
    """grad_leaf = sum_g J_g^T G[:, g, :] with each leaf's gradient taken in
    the game of its own tree's output; leaves in tree-major node-id order of
    the whole ensemble."""
    K, tg = _groups(ens)
    G = np.asarray(G, np.float64)
    assert G.shape[1] == K
    leaves_per_tree = np.array([int((ens.left[ens.tree_offsets[t]:ens.tree_offsets[t + 1]]
                                     < 0).sum()) for t in range(ens.n_trees)])
    first = np.concatenate([[0], np.cumsum(leaves_per_tree)])
    out = np.zeros(int(first[-1]))
    for g, trees in enumerate(tg):
        if not trees:
            continue
        part = leaf_grad(_sub(ens, trees), X, G[:, g, :], n, threads)
        pos = 0
        for t in trees:
            k = int(leaves_per_tree[t])
            out[first[t]:first[t] + k] = part[pos:pos + k]
            pos += k
    return out
