"""Seeded synthetic tree ensembles and explained samples.

This module is the single source of inputs shared by the oracle-side tests and
the GPU path.  It builds tree structure, thresholds, training-row covers, leaf
values and explained samples; it contains none of the Shapley / quadrature
arithmetic.

Model format (structure of arrays, node ids local to each tree, root = node 0):
  tree_offsets int64 [T+1]   node range of tree t is [tree_offsets[t], tree_offsets[t+1])
  left, right  int32 [N]     child ids local to the tree, -1 marks a leaf
  feature      int32 [N]     split feature (ignored at leaves)
  threshold    float32 [N]   a row goes left iff x < threshold (float32 compare)
  default_left uint8 [N]     direction of a missing (NaN) value
  cover        float64 [N]   number of training rows reaching the node
  value        float64 [N]   leaf value (ignored at internal nodes)

Two tree recipes, mirroring the growth regimes of the paper's benchmark table
(breadth-first full trees, and depth-first trees with a leaf cap):
  * random : every internal node draws a feature uniformly and a threshold that
    is a random quantile of N(0,1) (or, on integer-valued columns, an integer in
    1..9); a split that would leave a child without training rows is redrawn up
    to 32 times, after which the node becomes a leaf.  Grown breadth-first to
    the maximum depth.
  * grown  : depth-first, bigger child first, threshold = a U(0.05,0.95)
    quantile of the node's own training rows on a random feature, until the
    maximum depth, fewer than two rows, or the leaf cap.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
from scipy.special import ndtri

SEED_BASE = 2605_04497

_HERE = os.path.dirname(os.path.abspath(__file__))
_GROW_SRC = os.path.join(_HERE, "_grow.c")
_GROW_LIB = os.path.join(_HERE, "_grow.so")


@dataclass
class Ensemble:
    """A tree ensemble in the structure-of-arrays format described above."""

    tree_offsets: np.ndarray
    left: np.ndarray
    right: np.ndarray
    feature: np.ndarray
    threshold: np.ndarray
    default_left: np.ndarray
    cover: np.ndarray
    value: np.ndarray
    n_features: int
    base_score: float = 0.0
    meta: dict = field(default_factory=dict)
    # multi-output models: output group of every tree and the number of
    # groups (None: one output); base_score is then one value per group
    tree_group: np.ndarray | None = None
    n_groups: int = 1

    @property
    def n_trees(self) -> int:
        return int(self.tree_offsets.shape[0] - 1)

    @property
    def n_nodes(self) -> int:
        return int(self.left.shape[0])

    def leaf_mask(self) -> np.ndarray:
        return self.left < 0

    def n_leaves(self) -> int:
        return int(self.leaf_mask().sum())

    def leaf_values(self) -> np.ndarray:
        """Leaf values in tree-major, node-id order (the order of grad_leaf)."""
        return self.value[self.leaf_mask()].copy()

    def with_leaf_values(self, vals: np.ndarray) -> "Ensemble":
        v = self.value.copy()
        v[self.leaf_mask()] = np.asarray(vals, dtype=np.float64)
        return Ensemble(self.tree_offsets, self.left, self.right, self.feature,
                        self.threshold, self.default_left, self.cover, v,
                        self.n_features, self.base_score, dict(self.meta),
                        self.tree_group, self.n_groups)

    def with_groups(self, tree_group, n_groups: int, base_scores=None) -> "Ensemble":
        """The same trees as a multi-output model: tree t adds to output
        tree_group[t]; base_scores[g] is output g's bias (default 0)."""
        tg = np.ascontiguousarray(tree_group, np.int32)
        assert tg.shape == (self.n_trees,)
        bs = (np.zeros(n_groups) if base_scores is None
              else np.asarray(base_scores, np.float64).reshape(n_groups))
        return Ensemble(self.tree_offsets, self.left, self.right, self.feature,
                        self.threshold, self.default_left, self.cover, self.value,
                        self.n_features, bs, dict(self.meta), tg, int(n_groups))

    def group_trees(self, g: int) -> list:
        """Indices of the trees of output group g (all trees when ungrouped)."""
        if self.tree_group is None:
            return list(range(self.n_trees))
        return [int(t) for t in np.flatnonzero(self.tree_group == g)]

    def subset_trees(self, trees) -> "Ensemble":
        trees = list(trees)
        parts = {k: [] for k in ("left", "right", "feature", "threshold",
                                  "default_left", "cover", "value")}
        offs = [0]
        for t in trees:
            a, b = int(self.tree_offsets[t]), int(self.tree_offsets[t + 1])
            for k in parts:
                parts[k].append(getattr(self, k)[a:b])
            offs.append(offs[-1] + (b - a))
        cat = {k: np.concatenate(v) if v else np.zeros(0, getattr(self, k).dtype)
               for k, v in parts.items()}
        return Ensemble(np.asarray(offs, np.int64), cat["left"], cat["right"],
                        cat["feature"], cat["threshold"], cat["default_left"],
                        cat["cover"], cat["value"], self.n_features,
                        self.base_score, dict(self.meta))

    def stats(self) -> dict:
        """Realised max depth D, max unique-feature depth d and mean leaves."""
        D = 0
        d = 0
        for t in range(self.n_trees):
            a = int(self.tree_offsets[t])
            stack = [(0, 0, ())]
            while stack:
                node, depth, feats = stack.pop()
                g = a + node
                if self.left[g] < 0:
                    D = max(D, depth)
                    d = max(d, len(set(feats)))
                    continue
                f = int(self.feature[g])
                stack.append((int(self.left[g]), depth + 1, feats + (f,)))
                stack.append((int(self.right[g]), depth + 1, feats + (f,)))
        return {"trees": self.n_trees, "D": D, "d": d,
                "mean_leaves": self.n_leaves() / max(1, self.n_trees)}


def _concat_trees(trees, n_features, base_score=0.0, meta=None) -> Ensemble:
    offs = np.zeros(len(trees) + 1, np.int64)
    for i, t in enumerate(trees):
        offs[i + 1] = offs[i] + t["left"].shape[0]
    cat = {k: np.concatenate([t[k] for t in trees]) for k in trees[0]}
    return Ensemble(offs, cat["left"].astype(np.int32), cat["right"].astype(np.int32),
                    cat["feature"].astype(np.int32), cat["threshold"].astype(np.float32),
                    cat["default_left"].astype(np.uint8), cat["cover"].astype(np.float64),
                    cat["value"].astype(np.float64), int(n_features), float(base_score),
                    dict(meta or {}))


def normal_rows(rng, n, F, int_cols=()) -> np.ndarray:
    """Rows of N(0,1) float32; the listed columns hold uniform integers 0..9."""
    X = rng.standard_normal((n, F), dtype=np.float32)
    for c in int_cols:
        X[:, c] = rng.integers(0, 10, size=n).astype(np.float32)
    return X


def random_tree(rng, xt, depth, F, int_cols, sigma, max_tries=32) -> dict:
    """Breadth-first full-depth tree with random features and N(0,1) quantile
    thresholds.  xt is the training matrix transposed, [F, n_rows]."""
    n_rows = xt.shape[1]
    is_int = np.zeros(F, np.uint8)
    is_int[list(int_cols)] = 1
    max_inner = 2 ** depth - 1
    max_nodes = 2 ** (depth + 1) - 1
    n_c = max_inner * max_tries
    cf = rng.integers(0, F, size=n_c).astype(np.int32)
    cn = ndtri(rng.random(size=n_c)).astype(np.float32)
    ci = rng.integers(1, 10, size=n_c).astype(np.float32)
    rl = rng.integers(0, 2, size=max_inner).astype(np.uint8)
    out = _alloc_tree(max_nodes)
    P = ctypes.c_void_p
    n = _grow_lib().random_tree(
        P(xt.ctypes.data), ctypes.c_int64(n_rows), ctypes.c_int32(F),
        ctypes.c_int32(depth), P(is_int.ctypes.data), P(cf.ctypes.data),
        P(cn.ctypes.data), P(ci.ctypes.data), P(rl.ctypes.data),
        ctypes.c_int32(max_tries), ctypes.c_int64(max_inner), ctypes.c_int64(max_nodes),
        *[P(out[k].ctypes.data) for k in _TREE_KEYS])
    if n < 0:
        raise RuntimeError("random_tree: node budget exceeded")
    return _finish_tree(rng, out, n, sigma)


_TREE_KEYS = ("left", "right", "feature", "threshold", "default_left", "cover")


def _alloc_tree(max_nodes):
    return {"left": np.empty(max_nodes, np.int32), "right": np.empty(max_nodes, np.int32),
            "feature": np.empty(max_nodes, np.int32),
            "threshold": np.empty(max_nodes, np.float32),
            "default_left": np.empty(max_nodes, np.uint8),
            "cover": np.empty(max_nodes, np.float64)}


def _finish_tree(rng, out, n, sigma):
    out = {k: v[:n].copy() for k, v in out.items()}
    value = np.zeros(n, np.float64)
    leaves = out["left"] < 0
    value[leaves] = rng.normal(0.0, sigma, size=int(leaves.sum()))
    out["value"] = value
    return out


def _grow_lib():
    if (not os.path.exists(_GROW_LIB)
            or os.path.getmtime(_GROW_LIB) < os.path.getmtime(_GROW_SRC)):
        build_grow()
    lib = ctypes.CDLL(_GROW_LIB)
    lib.grow_tree.restype = ctypes.c_int64
    lib.random_tree.restype = ctypes.c_int64
    return lib


def build_grow() -> None:
    """Compile the depth-first grower (plain C, host only)."""
    tmp = _GROW_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _GROW_SRC])
    os.replace(tmp, _GROW_LIB)


def grown_tree(rng, xt, depth, leaf_cap, sigma) -> dict:
    F, n_rows = xt.shape
    max_nodes = int(min(2 * leaf_cap, 2 ** min(depth + 1, 40))) + 1
    rf = rng.integers(0, F, size=max_nodes).astype(np.int32)
    ru = rng.uniform(0.05, 0.95, size=max_nodes)
    rl = rng.integers(0, 2, size=max_nodes).astype(np.uint8)
    out = _alloc_tree(max_nodes)
    P = ctypes.c_void_p
    n = _grow_lib().grow_tree(
        P(xt.ctypes.data), ctypes.c_int64(n_rows), ctypes.c_int32(F),
        ctypes.c_int32(depth), ctypes.c_int64(leaf_cap), P(rf.ctypes.data),
        P(ru.ctypes.data), P(rl.ctypes.data), ctypes.c_int64(max_nodes),
        *[P(out[k].ctypes.data) for k in _TREE_KEYS])
    if n < 0:
        raise RuntimeError("grow_tree: node budget exceeded")
    return _finish_tree(rng, out, n, sigma)


# ----------------------------------------------------------------------------
# The five workloads.  Each takes overrides so tests can run scaled-down copies
# with the same structure.
# ----------------------------------------------------------------------------

CONFIGS = {
    # Plain FP64 SHAP values: 10 random trees of depth 4, 8 features.
    "c1_small": dict(index=0, kind="random", F=8, T=10, depth=4, n_train=10_000,
                     sigma=0.1, M=1000, int_frac=0.0),
    # SHAP values FP32 vs FP64: 1000 random trees of depth 8, 100 features,
    # 20 of them integer-valued.  The headline throughput workload.
    "c2_values": dict(index=1, kind="random", F=100, T=1000, depth=8, n_train=100_000,
                      sigma=0.05, M=100_000, int_frac=0.2),
    # Uneven depths 3..20 with pairwise interactions, 200 features.
    "c3_interactions": dict(index=2, kind="grown", F=200, T=500, depth=(3, 20),
                            leaf_cap=4096, n_train=100_000, sigma=0.05, M=50_000,
                            int_frac=0.0),
    # Adjoint to leaf values: 200 full random trees of depth 6 (12,800 leaves).
    "c4_adjoint": dict(index=3, kind="random_full", F=50, T=200, depth=6,
                       n_train=100_000, sigma=0.05, M=20_000, int_frac=0.0,
                       target_sigma=0.1),
    # Deep-tree stress: 100 grown trees of depth 32, leaf cap 512, 64 features.
    "c5_deep": dict(index=4, kind="grown", F=64, T=100, depth=32, leaf_cap=512,
                    n_train=200_000, sigma=0.05, M=10_000, int_frac=0.0),
}


@dataclass
class Workload:
    name: str
    ensemble: Ensemble
    X: np.ndarray
    target: np.ndarray | None
    cfg: dict


def make_workload(name: str, **over) -> Workload:
    """Build a seeded workload.  Overrides (T, M, n_train, depth, F, ...) give
    scaled-down copies; the seed depends only on the config index and the
    optional 'seed_offset' override.  groups=K makes a K-output model of the
    same trees (tree t adds to output t mod K)."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    seed = SEED_BASE + cfg["index"] + 1000 * int(cfg.get("seed_offset", 0))
    rng = np.random.default_rng(seed)
    F = cfg["F"]
    n_int = int(round(cfg.get("int_frac", 0.0) * F))
    int_cols = tuple(sorted(rng.choice(F, size=n_int, replace=False).tolist())) if n_int else ()
    Xtr = normal_rows(rng, cfg["n_train"], F, int_cols)
    xt = np.ascontiguousarray(Xtr.T)
    del Xtr
    trees = []
    kind = cfg["kind"]
    for _ in range(cfg["T"]):
        if kind == "random":
            trees.append(random_tree(rng, xt, cfg["depth"], F, int_cols, cfg["sigma"]))
        elif kind == "random_full":
            full = 2 ** cfg["depth"]
            for _attempt in range(100):
                t = random_tree(rng, xt, cfg["depth"], F, int_cols, cfg["sigma"])
                if int((t["left"] < 0).sum()) == full:
                    break
            else:
                raise RuntimeError("could not grow a full tree")
            trees.append(t)
        elif kind == "grown":
            dep = cfg["depth"]
            if isinstance(dep, tuple):
                dep = int(rng.integers(dep[0], dep[1] + 1))
            trees.append(grown_tree(rng, xt, dep, cfg["leaf_cap"], cfg["sigma"]))
        else:
            raise ValueError(kind)
    ens = _concat_trees(trees, F, 0.0, {"config": name, "int_cols": list(int_cols)})
    if cfg.get("groups", 1) > 1:
        # a multi-output model: boosting rounds add one tree per output in turn
        K = int(cfg["groups"])
        ens = ens.with_groups(np.arange(ens.n_trees) % K, K,
                              base_scores=0.5 - 0.25 * np.arange(K))
    X = normal_rows(rng, cfg["M"], F, int_cols)
    target = None
    if "target_sigma" in cfg:
        target = rng.normal(0.0, cfg["target_sigma"], size=(cfg["M"], F)).astype(np.float32)
    return Workload(name, ens, X, target, cfg)


def stump(n_left=30.0, n_right=70.0, v_left=1.0, v_right=-2.0, thr=0.0, F=1,
          feat=0, default_left=0) -> Ensemble:
    """One split on `feat`; used for closed-form pins."""
    return _concat_trees([{
        "left": np.array([1, -1, -1], np.int32), "right": np.array([2, -1, -1], np.int32),
        "feature": np.array([feat, 0, 0], np.int32),
        "threshold": np.array([thr, 0, 0], np.float32),
        "default_left": np.array([default_left, 0, 0], np.uint8),
        "cover": np.array([n_left + n_right, n_left, n_right], np.float64),
        "value": np.array([0.0, v_left, v_right], np.float64)}], F)


def from_nested(trees, n_features, base_score=0.0) -> Ensemble:
    """Build an ensemble from nested tuples, for hand-written test models.

    A leaf is ("leaf", value, cover); an internal node is
    ("split", feature, threshold, cover, left_subtree, right_subtree[, default_left]).
    """
    out = []
    for tree in trees:
        arr = {k: [] for k in ("left", "right", "feature", "threshold",
                                "default_left", "cover", "value")}

        def emit(node):
            i = len(arr["left"])
            for k in arr:
                arr[k].append(0)
            if node[0] == "leaf":
                arr["left"][i] = arr["right"][i] = -1
                arr["value"][i] = float(node[1])
                arr["cover"][i] = float(node[2])
                return i
            _, f, thr, cov, lt, rt, *rest = node
            arr["feature"][i] = int(f)
            arr["threshold"][i] = float(np.float32(thr))
            arr["cover"][i] = float(cov)
            arr["default_left"][i] = int(rest[0]) if rest else 0
            arr["left"][i] = emit(lt)
            arr["right"][i] = emit(rt)
            return i

        emit(tree)
        out.append({k: np.asarray(v) for k, v in arr.items()})
    return _concat_trees(out, n_features, base_score)


def random_small_ensemble(rng, n_trees, F, max_depth, n_train=200, sigma=1.0,
                          p_leaf=0.15, zero_cover=False) -> Ensemble:
    """Small irregular trees for brute-force checks: repeated features, uneven
    depth, integer ties.  With zero_cover some splits send no training rows to
    one child (a zero cover)."""
    Xtr = np.round(rng.standard_normal((n_train, F)).astype(np.float32) * 2) / 2
    trees = []
    for _ in range(n_trees):
        arr = {k: [] for k in ("left", "right", "feature", "threshold",
                                "default_left", "cover", "value")}

        def emit(rows, depth):
            i = len(arr["left"])
            for k in arr:
                arr[k].append(0)
            arr["cover"][i] = float(rows.shape[0])
            if depth >= max_depth or (depth > 0 and rng.random() < p_leaf):
                arr["left"][i] = arr["right"][i] = -1
                arr["value"][i] = float(rng.normal(0, sigma))
                return i
            if zero_cover and rng.random() < 0.2:
                f = int(rng.integers(F))
                thr = np.float32(100.0)  # every row goes left: right cover 0
                go = Xtr[rows, f] < thr
            else:
                for _ in range(32):
                    f = int(rng.integers(F))
                    thr = np.float32(np.round(rng.standard_normal() * 2) / 2)
                    go = Xtr[rows, f] < thr
                    if zero_cover or 0 < int(go.sum()) < rows.shape[0]:
                        break
                else:
                    arr["left"][i] = arr["right"][i] = -1
                    arr["value"][i] = float(rng.normal(0, sigma))
                    return i
            arr["feature"][i] = f
            arr["threshold"][i] = float(thr)
            arr["default_left"][i] = int(rng.integers(2))
            arr["left"][i] = emit(rows[go], depth + 1)
            arr["right"][i] = emit(rows[~go], depth + 1)
            return i

        emit(np.arange(n_train), 0)
        trees.append({k: np.asarray(v) for k, v in arr.items()})
    return _concat_trees(trees, F)
