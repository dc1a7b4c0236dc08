"""CPU tests of the host side of the library: the C-ABI exports, the
Gauss-Legendre rule, the collapsed path table, E[f] and model validation.
No GPU is used (ensembles are built with qts_build_host)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def q():
    import paper_2605_04497_amd as q
    return q


def test_library_exports_every_declared_symbol(q):
    header = open(os.path.join(ROOT, "include", "qtreeshap.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(qts_\w+)\s*\(", header, re.M))
    assert {"qts_load_ensemble", "qts_shap_values", "qts_shap_interactions",
            "qts_shap_backward", "qts_last_error"} <= declared
    lib = ctypes.CDLL(q._lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(q._lib.SIGNATURES) == declared


def test_gauss_legendre_rule(q, oracle_mod):
    """Golub-Welsch rule (library) vs Newton rule (oracle); both exact to degree 15."""
    for n in (1, 2, 5, 8, 16):
        t, s, w = q.gauss_legendre(n)
        t2, s2, w2 = oracle_mod.gauss_legendre(n)
        np.testing.assert_allclose(t, t2, atol=2e-15)
        np.testing.assert_allclose(s, s2, atol=2e-15)
        np.testing.assert_allclose(w, w2, rtol=5e-14)
        for k in range(2 * n):
            assert abs(np.sum(w * t ** k) - 1.0 / (k + 1)) < 1e-14 * (k + 1)
    t, s, w = q.gauss_legendre(8)
    assert np.all(np.diff(t) > 0) and np.all(t > 0) and np.all(s > 0)
    np.testing.assert_allclose(t[::-1], s, atol=1e-16)  # symmetric rule
    with pytest.raises(q.QtsError):
        q.gauss_legendre(0)


def test_fp32_rule_constants(q):
    """The FP32 walks over short rows take the 8-node rule as instruction
    literals (rule8_t32, rule8_w32 in the device header): they must be the
    FP32 rounding of the rule the library computes (Eq. 10), which the
    library also checks when it sets up a device."""
    src = open(os.path.join(ROOT, "paper_2605_04497_amd", "csrc", "qts_device.h")).read()

    def table(name):
        m = re.search(name + r"\(int m\) \{\s*constexpr float \w+\[kNodes\] = \{([^}]*)\}", src)
        assert m, name
        return np.array([float.fromhex(x.strip().rstrip("f")) for x in m.group(1).split(",")])

    t, s, w = q.gauss_legendre(8)
    assert np.array_equal(table("rule8_t32"), np.float32(t).astype(np.float64))
    assert np.array_equal(table("rule8_w32"), np.float32(w).astype(np.float64))


def _phi_from_table(tab, leaf_values, X, F):
    """Re-evaluate phi from the exported table in numpy (test-only path form)."""
    x, wq = np.polynomial.legendre.leggauss(8)
    t, w = (1 + x) / 2, wq / 2
    M = X.shape[0]
    phi = np.zeros((M, F))
    for p in range(tab["path_len"].shape[0]):
        a, d = tab["path_off"][p], tab["path_len"][p]
        f = tab["feat"][a:a + d]
        lo, hi, mok = tab["lo"][a:a + d], tab["hi"][a:a + d], tab["missing_ok"][a:a + d] != 0
        b, cb = tab["b"][a:a + d], tab["one_minus_b"][a:a + d]
        xv = X[:, f]
        with np.errstate(invalid="ignore"):
            inside = (xv >= lo) & (np.isnan(hi) | (xv < hi))
        o = np.where(np.isnan(xv), mok, inside).astype(float)          # [M, d]
        fac = b[None, :, None] * (1 - t) + o[:, :, None] * t           # [M, d, 8]
        val = leaf_values[tab["path_leaf"][p]]
        for j in range(d):
            loo = np.prod(np.delete(fac, j, axis=1), axis=1)            # [M, 8]
            coef = np.where(o[:, j] > 0, cb[j], -b[j])
            phi[:, f[j]] += val * coef * (loo @ w)
    return phi


@pytest.mark.parametrize("name,over", [
    ("c1_small", dict(M=40)),
    ("c2_values", dict(T=4, M=30, n_train=4000)),
    ("c5_deep", dict(T=3, M=12, n_train=20000)),
])
def test_path_table_reproduces_oracle(q, oracle_mod, name, over):
    wl = synth.make_workload(name, **over)
    ens, X = wl.ensemble, wl.X.copy()
    X[0, :] = np.nan
    X[1, ::3] = np.nan
    e = q.Ensemble(ens, host_only=True)
    tab = e.export_paths()
    assert e.info["device"] == -1 and e.n_leaves == ens.n_leaves()
    assert e.info["max_unique"] <= e.info["max_depth"]
    np.testing.assert_allclose(tab["b"] + tab["one_minus_b"], 1.0, atol=1e-15)
    phi = _phi_from_table(tab, ens.leaf_values(), X, ens.n_features)
    want = oracle_mod.shap_values(ens, X, n=8)
    np.testing.assert_allclose(phi, want, atol=1e-12 * max(1.0, np.abs(want).max()))
    assert e.expected_value == pytest.approx(oracle_mod.expected_value(ens), abs=1e-13)


def test_expected_value_includes_base_score(q, oracle_mod):
    ens = synth.stump()
    ens.base_score = 0.25
    e = q.Ensemble(ens, host_only=True)
    assert e.expected_value == pytest.approx(-1.1 + 0.25, abs=1e-15)


def test_single_leaf_tree_and_null_default_left(q):
    ens = synth.from_nested([("leaf", 3.0, 10.0), ("split", 0, 0.0, 10.0, ("leaf", 1.0, 4.0),
                                                   ("leaf", 2.0, 6.0))], n_features=1)
    e = q.Ensemble(ens, host_only=True)
    assert e.n_leaves == 3 and e.info["n_paths"] == 2
    assert e.expected_value == pytest.approx(3.0 + 0.4 + 1.2)
    # default_left = NULL means every missing value goes right
    L = q._lib
    a = {k: np.ascontiguousarray(getattr(ens, k)) for k in (
        "tree_offsets", "left", "right", "feature", "threshold", "cover", "value")}
    ta = L.TreeArrays(ens.n_trees, a["tree_offsets"].ctypes.data, a["left"].ctypes.data,
                      a["right"].ctypes.data, a["feature"].ctypes.data,
                      a["threshold"].ctypes.data, None, a["cover"].ctypes.data,
                      a["value"].ctypes.data)
    h = ctypes.c_void_p()
    L.check(L.lib().qts_build_host(ctypes.byref(ta), 1, 0.0, ctypes.byref(h)))
    mok = np.zeros(2, np.uint8)
    L.check(L.lib().qts_export_paths(h, None, None, None, None, None, None,
                                     mok.ctypes.data, None, None))
    assert list(mok) == [0, 1]  # left path: NaN goes right -> not ok; right path ok
    L.check(L.lib().qts_free_ensemble(h))


def _arrays(**over):
    base = dict(tree_offsets=[0, 3], left=[1, -1, -1], right=[2, -1, -1], feature=[0, 0, 0],
                threshold=[0.0, 0.0, 0.0], default_left=[0, 0, 0], cover=[10.0, 4.0, 6.0],
                value=[0.0, 1.0, 2.0])
    base.update(over)
    return synth.Ensemble(np.asarray(base["tree_offsets"], np.int64),
                          np.asarray(base["left"], np.int32), np.asarray(base["right"], np.int32),
                          np.asarray(base["feature"], np.int32),
                          np.asarray(base["threshold"], np.float32),
                          np.asarray(base["default_left"], np.uint8),
                          np.asarray(base["cover"], np.float64),
                          np.asarray(base["value"], np.float64), base.get("F", 2))


@pytest.mark.parametrize("over,code", [
    (dict(left=[1, 1, -1]), -2),                      # node reached twice
    (dict(left=[0, -1, -1]), -2),                     # cycle back to the root
    (dict(left=[1, -1, -1], right=[-1, -1, -1]), -2),  # one child
    (dict(left=[5, -1, -1]), -2),                     # child out of range
    (dict(feature=[2, 0, 0]), -2),                    # feature >= F
    (dict(feature=[-1, 0, 0]), -2),
    (dict(cover=[10.0, -1.0, 6.0]), -2),              # negative cover
    (dict(cover=[10.0, np.nan, 6.0]), -2),            # NaN cover
    (dict(threshold=[np.nan, 0.0, 0.0]), -2),         # NaN threshold
    (dict(tree_offsets=[0, 0]), -2),                  # empty tree
    (dict(tree_offsets=[1, 3]), -2),
    (dict(F=0), -1),                                  # no features
])
def test_invalid_models_are_rejected(q, over, code):
    with pytest.raises(q.QtsError) as ei:
        q.Ensemble(_arrays(**over), host_only=True)
    assert ei.value.code == code
    assert len(q._lib.lib().qts_last_error()) > 0


def _chain(depth, n_features, distinct=True):
    node = ("leaf", 1.0, 1.0)
    for j in reversed(range(depth)):
        node = ("split", j if distinct else 0, 0.0, 2.0, node, ("leaf", 0.0, 1.0))
    return synth.from_nested([node], n_features=n_features)


def test_limits(q):
    q.Ensemble(_chain(64, 64), host_only=True)          # 64 unique features: fine
    with pytest.raises(q.QtsError) as ei:
        q.Ensemble(_chain(65, 65), host_only=True)      # 65 unique features
    assert ei.value.code == -3
    e = q.Ensemble(_chain(128, 1, distinct=False), host_only=True)
    assert e.info["max_depth"] == 128 and e.info["max_unique"] == 1
    with pytest.raises(q.QtsError) as ei:
        q.Ensemble(_chain(129, 1, distinct=False), host_only=True)
    assert ei.value.code == -3


def test_null_arguments_and_host_only_compute(q):
    L = q._lib
    h = ctypes.c_void_p()
    assert L.lib().qts_build_host(None, 1, 0.0, ctypes.byref(h)) == -1
    assert L.lib().qts_expected_value(None, None) == -1
    assert L.lib().qts_free_ensemble(None) == 0
    e = q.Ensemble(synth.stump(), host_only=True)
    rc = L.lib().qts_shap_values(e._h, None, 0, 1, None, None, 0, None)
    assert rc == -1  # host-only ensembles cannot compute
    assert b"host-only" in L.lib().qts_last_error()
    rc = L.lib().qts_shap_values(e._h, None, -1, 1, None, None, 0, None)
    assert rc == -1
    rc = L.lib().qts_shap_values(e._h, None, 1, 0, None, None, 0, None)
    assert rc == -1  # ldx < F
    rc = L.lib().qts_shap_values(e._h, None, 0, 1, None, None, 7, None)
    assert rc == -1  # unknown precision


@pytest.mark.parametrize("name,over", [
    ("c1_small", dict(M=4)),
    ("c3_interactions", dict(T=6, M=4, n_train=20000)),
    ("c5_deep", dict(T=3, M=4, n_train=30000)),
])
def test_sibling_merge_counts(q, name, over):
    """The first-order table merges exactly the pairs of leaves that are the
    two children of one node (a node whose children are both leaves), and
    keeps every other path."""
    wl = synth.make_workload(name, **over)
    ens = wl.ensemble
    left, right = np.asarray(ens.left), np.asarray(ens.right)
    offs = np.asarray(ens.tree_offsets)
    want = 0
    for t in range(ens.n_trees):
        a, b = offs[t], offs[t + 1]
        lt, rt = left[a:b], right[a:b]
        inner = lt >= 0
        want += int(np.sum(inner & (lt[np.maximum(lt, 0)] < 0) & (lt[np.maximum(rt, 0)] < 0)))
    e = q.Ensemble(ens, host_only=True)
    info = e.info
    assert info["n_merged"] == want
    assert info["n_value_paths"] == info["n_paths"] - want
    # a merged pair has one row of the same length as each of its two paths
    d = e.export_paths()["path_len"]
    assert info["n_value_elements"] <= info["n_elements"]
    assert info["n_elements"] - info["n_value_elements"] >= want   # each pair drops >= 1 element
    assert d.min() >= 1


def _first_order_rows(ens, merged):
    """Rows of the first-order table rebuilt from the trees (independently of
    the library): per leaf with at least one split, its unique features in
    order of first appearance with (feature, missing_ok, lo, hi, b); two leaf
    children of one node with the same feature count form one merged row with
    the parent's split feature in slot 0; a single path puts its deepest
    feature in slot 0 (merged table) or keeps path order (unmerged table).
    Rows are in tree and left-to-right leaf order, stably grouped by length
    capacity 8, 16, 32, 64."""
    left, right = np.asarray(ens.left), np.asarray(ens.right)
    feat, thr = np.asarray(ens.feature), np.asarray(ens.threshold, dtype=np.float32)
    dleft, cover = np.asarray(ens.default_left), np.asarray(ens.cover, dtype=np.float64)
    offs = np.asarray(ens.tree_offsets)
    paths = []   # (elements dict in first-appearance order, parent node, is_left, tree)
    for t in range(ens.n_trees):
        a = int(offs[t])

        def walk(node, edges):
            g = a + node
            if left[g] < 0:
                el = {}
                for (f, is_left, th, dl, w, _) in edges:
                    lo, hi, mok, b = el.get(f, (-np.inf, None, True, 1.0))
                    b = b * w
                    if is_left:
                        hi = th if hi is None else min(hi, th)
                        mok = mok and bool(dl)
                    else:
                        lo = max(lo, th)
                        mok = mok and not bool(dl)
                    el[f] = (lo, hi, mok, b)
                if el:
                    parent = edges[-1][5] if edges else -1
                    paths.append(([(f,) + v for f, v in el.items()], parent, edges[-1][1], t))
                return
            cp = cover[g]
            for child, is_left in ((int(left[g]), True), (int(right[g]), False)):
                w = 0.0 if cp == 0.0 else cover[a + child] / cp
                walk(child, edges + [(int(feat[g]), is_left, thr[g], dleft[g], w, node)])

        walk(0, [])
    rows = []
    i = 0
    while i < len(paths):
        A = paths[i]
        if merged and i + 1 < len(paths):
            B = paths[i + 1]
            if (A[1] >= 0 and A[1] == B[1] and A[3] == B[3] and A[2] and not B[2]
                    and len(A[0]) == len(B[0])):
                L = int(feat[int(offs[A[3]]) + A[1]])
                kL = [e[0] for e in A[0]].index(L)
                rows.append([A[0][kL]] + A[0][:kL] + A[0][kL + 1:])
                i += 2
                continue
        rows.append(A[0][-1:] + A[0][:-1] if merged else A[0])
        i += 1
    cap = lambda d: min(c for c in (8, 16, 32, 64) if d <= c)
    return sorted(rows, key=lambda r: cap(len(r)))


def _shared_slots(rows):
    total = 0
    for prev, row in zip(rows, rows[1:]):
        k = 1
        while k < min(len(prev), len(row)) and prev[k] == row[k]:
            k += 1
        total += k - 1
    return total


@pytest.mark.parametrize("name,over", [
    ("c1_small", dict(M=4)),
    ("c2_values", dict(T=12, M=4, n_train=20000)),
    ("c3_interactions", dict(T=6, M=4, n_train=20000)),
    ("c5_deep", dict(T=2, M=4, n_train=30000)),
])
def test_shared_prefix_counts(q, name, over):
    """The first-order kernels reuse the work of the leading slots (after slot
    0) that equal the previous row's; the library's per-table totals must
    equal those of the rows rebuilt here (rows of every length)."""
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble, host_only=True)
    want_m = _shared_slots(_first_order_rows(wl.ensemble, merged=True))
    want_p = _shared_slots(_first_order_rows(wl.ensemble, merged=False))
    assert e.info["n_value_shared"] == want_m
    assert e.info["n_path_shared"] == want_p
    if name == "c2_values":
        assert want_m > 0 and want_p > 0


def test_shared_prefix_stops_at_first_difference(q):
    """Hand-made tree: the root splits on f0; its left child on f1, whose left
    child splits on f2 and whose right child splits on f0 again."""
    tree = ("split", 0, 0.0, 100.0,
            ("split", 1, 1.0, 60.0,
             ("split", 2, 2.0, 30.0, ("leaf", 1.0, 10.0), ("leaf", 2.0, 20.0)),
             ("split", 0, -1.0, 30.0, ("leaf", 3.0, 15.0), ("leaf", 4.0, 15.0))),
            ("leaf", 5.0, 40.0))
    ens = synth.from_nested([tree], n_features=3)
    e = q.Ensemble(ens, host_only=True)
    rows = _first_order_rows(ens, merged=True)
    assert len(rows) == 3 and e.info["n_merged"] == 2
    # merged rows: [f2 | f0, f1], [f0 narrowed to x < -1 | f1 right], [f0
    # right]: slot 1 holds f0 then f1, nothing is shared
    assert e.info["n_value_shared"] == _shared_slots(rows) == 0
    # unmerged rows: [f0, f1 left, f2 left], [f0, f1 left, f2 right] share
    # slot 1; [f0 narrowed, f1 right] differs from it in slot 1; [f0 in
    # [-1, 0), f1 right] shares slot 1 with it; the root's right leaf has
    # no slot after 0
    assert e.info["n_path_shared"] == _shared_slots(_first_order_rows(ens, merged=False)) == 2


def test_wide_feature_space_segments(q):
    """Beyond 210 features the first-order table is cut into segments of rows
    using at most 96 distinct features (the LDS tile of one work item); a
    table of every feature fits below that, and has none."""
    wl = synth.make_workload("c2_values", F=784, T=12, M=4, n_train=20000)
    e = q.Ensemble(wl.ensemble, host_only=True)
    n_seg = e.info["n_value_segments"]
    assert n_seg > 0
    # each segment holds whole rows and at most 96 features: at least
    # (distinct features of the table) / 96 segments
    used = len(set(wl.ensemble.feature[wl.ensemble.left >= 0].tolist()))
    assert n_seg >= -(-used // 96)
    for F in (100, 210):
        wl = synth.make_workload("c2_values", F=F, T=4, M=4, n_train=20000)
        assert q.Ensemble(wl.ensemble, host_only=True).info["n_value_segments"] == 0
    wl = synth.make_workload("c2_values", F=211, T=4, M=4, n_train=20000)
    assert q.Ensemble(wl.ensemble, host_only=True).info["n_value_segments"] > 0
