"""GPU parity of qts_shap_values against the FP64 oracle (8-node rule), on the
shapes of the five workloads scaled down, on sampled rows of the full-size
headline workload in the benchmark's launch configuration, and on edge cases."""
import functools

import numpy as np
import pytest

import synth
from tests.parity import check, row_normwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@functools.lru_cache(maxsize=2)
def _full_c2():
    return synth.make_workload("c2_values")


@pytest.fixture(scope="module")
def q():
    import paper_2605_04497_amd as q
    return q


def _run(q, ens, X, precision, leaf_values=None):
    e = q.Ensemble(ens)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lv = None if leaf_values is None else torch.from_numpy(leaf_values).cuda()
    phi = e.shap_values(Xd, precision, leaf_values=lv)
    torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64), e


CASES = [
    ("c1_small", dict()),                                   # whole workload
    ("c2_values", dict(T=40, M=333, n_train=20000)),        # ragged tail, int ties
    ("c3_interactions", dict(T=6, M=130, n_train=20000)),   # depths 3..20: buckets 8/16/32
    ("c4_adjoint", dict(T=20, M=200, n_train=20000)),
    ("c5_deep", dict(T=4, M=70, n_train=30000)),            # d up to ~30
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_values_match_oracle(q, oracle_mod, name, over, precision):
    print("case", name, over, precision, flush=True)
    wl = synth.make_workload(name, **over)
    got, e = _run(q, wl.ensemble, wl.X, precision)
    want = oracle_mod.shap_values(wl.ensemble, wl.X, n=8)
    check(got, want, precision, name)
    # efficiency (exact only where the 8-node rule is exact: d <= 16)
    if e.info["max_unique"] <= 16:
        fx = oracle_mod.predict(wl.ensemble, wl.X)
        res = np.abs(got.sum(1) + e.expected_value - fx).max()
        scale = max(1.0, np.abs(fx).max())
        assert res <= (1e-4 if precision == "fp32" else 1e-10) * scale


def test_c1_fp64_matches_enumeration(q):
    """FP64 GPU vs subset enumeration of the Shapley definition (F = 8)."""
    from oracle import brute
    wl = synth.make_workload("c1_small", M=24)
    got, _ = _run(q, wl.ensemble, wl.X, "fp64")
    assert row_normwise(got, brute.shap_values(wl.ensemble, wl.X)) <= 1e-10


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_headline_sampled_rows(q, oracle_mod, precision):
    """The benchmark's workload at full size (1000 trees, 100k samples, same
    launch configuration), checked on seeded sampled rows."""
    print("full-size c2_values", precision, flush=True)
    wl = _full_c2()
    got, e = _run(q, wl.ensemble, wl.X, precision)
    rows = np.random.default_rng(5).choice(wl.X.shape[0], 24, replace=False)
    rows = np.concatenate([rows, [0, 63, 64, wl.X.shape[0] - 1]])
    want = oracle_mod.shap_values(wl.ensemble, wl.X[rows], n=8)
    check(got[rows], want, precision, "c2 full")
    fx = oracle_mod.predict(wl.ensemble, wl.X[rows])
    assert np.abs(got[rows].sum(1) + e.expected_value - fx).max() <= 1e-4 * max(
        1.0, np.abs(fx).max())


def test_edge_cases(q, oracle_mod):
    wl = synth.make_workload("c4_adjoint", T=5, M=130, n_train=5000)
    ens, X = wl.ensemble, wl.X.copy()
    X[3, :] = np.nan
    X[5, ::2] = np.nan
    X[7, 1] = np.inf
    X[8, 2] = -np.inf
    e = q.Ensemble(ens)
    # M = 0 is a no-op
    out = e.shap_values(torch.zeros((0, ens.n_features), device="cuda"))
    assert out.shape == (0, ens.n_features)
    for precision in ("fp32", "fp64"):
        want = oracle_mod.shap_values(ens, X, n=8)
        Xd = torch.from_numpy(X).cuda()
        got = e.shap_values(Xd, precision).cpu().numpy()
        check(got, want, precision, "nan/inf rows")
        # single row, and a row stride larger than F
        got1 = e.shap_values(Xd[7:8], precision).cpu().numpy()
        check(got1, want[7:8], precision, "M=1")
        wide = torch.zeros((X.shape[0], ens.n_features + 9), device="cuda")
        wide[:, :ens.n_features] = Xd
        got_w = e.shap_values(wide[:, :ens.n_features], precision).cpu().numpy()
        check(got_w, want, precision, "ldx > F")


def test_leaf_value_override_and_linearity(q, oracle_mod):
    wl = synth.make_workload("c2_values", T=10, M=100, n_train=5000)
    ens = wl.ensemble
    rng = np.random.default_rng(9)
    v = rng.normal(size=ens.n_leaves())
    want = oracle_mod.shap_values(ens.with_leaf_values(v), wl.X)
    for precision in ("fp32", "fp64"):
        got, _ = _run(q, ens, wl.X, precision, leaf_values=v)
        check(got, want, precision, "leaf override")


def test_zero_covers_and_repeated_features(q, oracle_mod):
    for seed in range(3):
        rng = np.random.default_rng(300 + seed)
        ens = synth.random_small_ensemble(rng, 6, 7, 7, zero_cover=True)
        X = (np.round(rng.standard_normal((90, 7)) * 2) / 2).astype(np.float32)
        X[::7, 2] = np.nan
        want = oracle_mod.shap_values(ens, X, n=8)
        for precision in ("fp32", "fp64"):
            got, _ = _run(q, ens, X, precision)
            check(got, want, precision, "zero covers")


def chain_model(d, b=0.5):
    """A chain of d distinct features; every left branch continues (cover ratio
    b), every right branch is a leaf whose value varies with its depth."""
    node = ("leaf", 1.0, b ** d)
    for j in reversed(range(d)):
        val = (0.2 + 0.05 * (j % 7)) * (-1) ** j
        node = ("split", j, 0.0, b ** j, node, ("leaf", val, b ** j * (1 - b)))
    return synth.from_nested([node], n_features=d + 1)


def chain_rows(d):
    X = np.full((3, d + 1), -1.0, np.float32)
    X[1, d // 2] = 1.0   # leaves the chain half way
    X[2, :] = np.nan     # missing everywhere: goes right at the root
    return X


@pytest.mark.parametrize("d", [1, 8, 9, 16, 17, 24, 25, 31, 32, 33, 48, 64])
def test_bucket_boundaries_chain(q, oracle_mod, d):
    """Every bucket capacity and batch count at and around its boundaries
    (paths padded to whole batches of eight), against the oracle's 8-node
    value (exact for d <= 16)."""
    ens, X = chain_model(d), chain_rows(d)
    want = oracle_mod.shap_values(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        got, _ = _run(q, ens, X, precision)
        check(got, want, precision, "chain d=%d" % d)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_sibling_merge_matches_unmerged(q, oracle_mod, name, over, precision):
    """The merged first-order table (one row per pair of sibling leaves) and
    the plain one (one row per leaf) give the oracle's values."""
    print("case", name, over, precision, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    assert e.info["n_merged"] > 0
    X = torch.from_numpy(wl.X).cuda()
    merged = e.shap_values(X, precision).double().cpu().numpy()
    e.set_sibling_merge(False)
    plain = e.shap_values(X, precision).double().cpu().numpy()
    e.set_sibling_merge(True)
    want = oracle_mod.shap_values(wl.ensemble, wl.X, n=8)
    check(merged, want, precision, name + " merged")
    check(plain, want, precision, name + " plain")


def _sibling_leaf_pairs(ens):
    """(left, right) leaf ordinals of every node whose two children are leaves."""
    left, right = np.asarray(ens.left), np.asarray(ens.right)
    offs = np.asarray(ens.tree_offsets)
    pairs, base = [], 0
    for t in range(ens.n_trees):
        a, b = offs[t], offs[t + 1]
        lt, rt = left[a:b], right[a:b]
        is_leaf = lt < 0
        ordinal = np.cumsum(is_leaf) - 1 + base
        for v in np.nonzero(~is_leaf)[0]:
            if is_leaf[lt[v]] and is_leaf[rt[v]]:
                pairs.append((ordinal[lt[v]], ordinal[rt[v]]))
        base += int(is_leaf.sum())
    return pairs


def test_sibling_merge_cancellation_and_overrides(q, oracle_mod):
    """Sibling leaves with equal and opposite values (the combined factor's
    constant term cancels), equal values, one zero value, zero covers and
    NaN rows, through the model's leaf values and through an override."""
    for seed in range(3):
        rng = np.random.default_rng(700 + seed)
        ens = synth.random_small_ensemble(rng, 8, 7, 6, zero_cover=(seed == 2))
        v = ens.leaf_values().copy()
        pairs = _sibling_leaf_pairs(ens)
        assert pairs
        for n, (a, b) in enumerate(pairs):
            if n % 3 == 0:
                v[b] = -v[a]
            elif n % 3 == 1:
                v[b] = v[a]
            else:
                v[a] = 0.0
        X = (np.round(rng.standard_normal((75, 7)) * 2) / 2).astype(np.float32)
        X[::5, 3] = np.nan
        X[11, :] = np.nan
        want = oracle_mod.shap_values(ens.with_leaf_values(v), X, n=8)
        for precision in ("fp32", "fp64"):
            got, _ = _run(q, ens.with_leaf_values(v), X, precision)
            check(got, want, precision, "sibling values")
            got, _ = _run(q, ens, X, precision, leaf_values=v)
            check(got, want, precision, "sibling values via override")


@pytest.mark.parametrize("name,over", [
    ("c2_values", dict(T=40, M=333, n_train=20000)),      # every path d <= 8: 4 nodes
    ("c5_deep", dict(T=4, M=70, n_train=30000)),          # longer buckets keep 8 nodes
    ("c4_adjoint", dict(T=20, M=200, n_train=20000)),
])
def test_exact_node_policy(q, oracle_mod, name, over):
    """With the 'exact' node policy, paths of at most 8 features use 4 nodes;
    their integrands have degree <= 7, so the values equal the 8-node ones
    (and the 4-node oracle's) up to rounding, and so does the adjoint."""
    print("case", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    e.set_node_policy("exact")
    X = torch.from_numpy(wl.X).cuda()
    want = oracle_mod.shap_values(wl.ensemble, wl.X, n=8)
    G = np.random.default_rng(3).normal(size=want.shape)
    want_g = oracle_mod.leaf_grad(wl.ensemble, wl.X, G)
    for precision in ("fp32", "fp64"):
        got = e.shap_values(X, precision).double().cpu().numpy()
        check(got, want, precision, name + " exact nodes")
        Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
        g = e.shap_backward(X, torch.from_numpy(Gp).cuda(), precision).cpu().numpy()
        wg = oracle_mod.leaf_grad(wl.ensemble, wl.X, Gp) if precision == "fp32" else want_g
        err = np.abs(g - wg).max() / np.abs(wg).max()
        assert err <= (1e-5 if precision == "fp32" else 1e-10), err
    if e.info["max_unique"] <= 8:
        check(got, oracle_mod.shap_values(wl.ensemble, wl.X, n=4), "fp64", "4-node oracle")


@pytest.mark.parametrize("M", [1, 63, 300, 2000])
def test_shared_prefix_walk(q, oracle_mod, M):
    """Rows of at most 8 features (FP32) reuse the factors of the leading slots
    they share with the previous row; each wave's run of rows starts afresh.
    The sample count moves the chunk boundaries (and so where runs start);
    NaN inputs take the missing-value path; both tables and both node rules;
    a leaf-value override changes the folded slot-0 factor only."""
    print("case shared prefix M =", M, flush=True)
    wl = synth.make_workload("c2_values", T=25, M=M, n_train=20000)
    ens = wl.ensemble
    X = wl.X.copy()
    rng = np.random.default_rng(M)
    X[rng.random(X.shape) < 0.05] = np.nan
    lv = rng.normal(size=ens.n_leaves())
    want = oracle_mod.shap_values(ens, X, n=8)
    want_lv = oracle_mod.shap_values(ens.with_leaf_values(lv), X, n=8)
    e = q.Ensemble(ens)
    assert e.info["n_value_shared"] > 0
    Xd = torch.from_numpy(X).cuda()
    lvd = torch.from_numpy(lv).cuda()
    for merge in (True, False):
        e.set_sibling_merge(merge)
        for policy in ("fixed8", "exact"):
            e.set_node_policy(policy)
            tag = "merge=%s %s" % (merge, policy)
            got = e.shap_values(Xd, "fp32").double().cpu().numpy()
            check(got, want, "fp32", "shared prefix " + tag)
            got = e.shap_values(Xd, "fp32", leaf_values=lvd).double().cpu().numpy()
            check(got, want_lv, "fp32", "shared prefix, leaf override " + tag)


def _with_single_leaf_trees(ens, every, value):
    """The ensemble with a single-leaf tree (an empty path) after every
    `every`-th tree and before the first."""
    trees = []
    for t in range(ens.n_trees):
        if t % every == 0:
            trees.append(None)
        trees.append(t)
    parts = {k: [] for k in ("left", "right", "feature", "threshold", "default_left", "cover",
                              "value")}
    offs = [0]
    for t in trees:
        if t is None:
            one = {"left": [-1], "right": [-1], "feature": [0], "threshold": [0.0],
                   "default_left": [0], "cover": [100.0], "value": [value]}
            for k in parts:
                parts[k].append(np.asarray(one[k], dtype=getattr(ens, k).dtype))
            offs.append(offs[-1] + 1)
            continue
        a, b = int(ens.tree_offsets[t]), int(ens.tree_offsets[t + 1])
        for k in parts:
            parts[k].append(getattr(ens, k)[a:b])
        offs.append(offs[-1] + (b - a))
    cat = {k: np.concatenate(v) for k, v in parts.items()}
    return synth.Ensemble(np.asarray(offs, np.int64), cat["left"], cat["right"], cat["feature"],
                          cat["threshold"], cat["default_left"], cat["cover"], cat["value"],
                          ens.n_features, ens.base_score, dict(ens.meta))


@pytest.mark.parametrize("M", [5, 130])
def test_short_rows_with_empty_paths(q, oracle_mod, M):
    """Single-leaf trees give rows without features among the rows of at most
    8 features: the walk over short rows takes them like any row (they add
    nothing), and the row after one starts its shared prefix afresh; both
    tables, both node rules, both precisions, NaN inputs."""
    print("case empty paths M =", M, flush=True)
    wl = synth.make_workload("c2_values", T=12, M=M, n_train=20000)
    ens = _with_single_leaf_trees(wl.ensemble, 3, 2.5)
    X = wl.X.copy()
    rng = np.random.default_rng(900 + M)
    X[rng.random(X.shape) < 0.05] = np.nan
    want = oracle_mod.shap_values(ens, X, n=8)
    e = q.Ensemble(ens)
    Xd = torch.from_numpy(X).cuda()
    for merge in (True, False):
        e.set_sibling_merge(merge)
        for policy in ("fixed8", "exact"):
            e.set_node_policy(policy)
            for precision in ("fp32", "fp64"):
                tag = "empty paths merge=%s %s %s" % (merge, policy, precision)
                got = e.shap_values(Xd, precision).double().cpu().numpy()
                check(got, want, precision, tag)
    fx = oracle_mod.predict(ens, X)
    got = e.shap_values(Xd, "fp64").cpu().numpy()
    assert np.abs(got.sum(1) + e.expected_value - fx).max() <= 1e-10 * max(1.0, np.abs(fx).max())
    # the adjoint walks the same rows: the single leaves' gradients are 0
    G = rng.normal(size=(M, ens.n_features))
    single = np.flatnonzero(np.diff(ens.tree_offsets) == 1)
    for precision, tol in (("fp32", 1e-5), ("fp64", 1e-10)):
        Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
        want = oracle_mod.leaf_grad(ens, X, Gp)
        Gd = torch.from_numpy(Gp).cuda()
        if precision == "fp32":
            Gd = Gd.float()
        for merge in (True, False):
            e.set_sibling_merge(merge)
            for policy in ("fixed8", "exact"):
                e.set_node_policy(policy)
                for det in (False, True):
                    e.set_deterministic(det)
                    g = e.shap_backward(Xd, Gd, precision).cpu().numpy()
                    err = np.linalg.norm(g - want) / np.linalg.norm(want)
                    assert err <= tol, (precision, merge, policy, det, err)
                    leaf_ids = np.cumsum(ens.leaf_mask()) - 1
                    assert np.all(g[leaf_ids[ens.tree_offsets[single]]] == 0.0)
        e.set_deterministic(False)


@pytest.mark.parametrize("M", [1, 77, 700])
def test_long_row_reuse(q, oracle_mod, M):
    """Rows of more than 8 features (deep grown trees, buckets 16, 32 and 64)
    reuse the c_j of the leading slots they share with the previous row and,
    with all nodes in one pass, the prefix checkpoints of whole shared
    batches; each wave's run of rows starts afresh.  The sample count moves
    the chunk boundaries; NaN inputs, both tables, FP32 and FP64 (two node
    passes: no checkpoint reuse), and a leaf-value override."""
    print("case long-row reuse M =", M, flush=True)
    wl = synth.make_workload("c5_deep", T=4, M=M, n_train=30000)
    ens = wl.ensemble
    X = wl.X.copy()
    rng = np.random.default_rng(900 + M)
    X[rng.random(X.shape) < 0.05] = np.nan
    lv = rng.normal(size=ens.n_leaves())
    want = oracle_mod.shap_values(ens, X, n=8)
    want_lv = oracle_mod.shap_values(ens.with_leaf_values(lv), X, n=8)
    e = q.Ensemble(ens)
    assert e.info["max_unique"] > 16 and e.info["n_value_shared"] > 0
    Xd = torch.from_numpy(X).cuda()
    lvd = torch.from_numpy(lv).cuda()
    for merge in (True, False):
        e.set_sibling_merge(merge)
        for precision in ("fp32", "fp64"):
            tag = "merge=%s %s" % (merge, precision)
            got = e.shap_values(Xd, precision).double().cpu().numpy()
            check(got, want, precision, "long rows " + tag)
            got = e.shap_values(Xd, precision, leaf_values=lvd).double().cpu().numpy()
            check(got, want_lv, precision, "long rows, leaf override " + tag)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_output_fully_overwritten(q, oracle_mod, precision):
    """Calls that write phi directly from the workgroups (one bucket walked
    as one chunk: a small table) and calls that accumulate and cast must both
    overwrite every entry of an `out=` buffer that holds garbage."""
    for name, over in (("c1_small", dict(M=333)), ("c5_deep", dict(T=2, M=70, n_train=30000))):
        print("case", name, precision, flush=True)
        wl = synth.make_workload(name, **over)
        e = q.Ensemble(wl.ensemble)
        X = torch.from_numpy(wl.X).cuda()
        dt = torch.float32 if precision == "fp32" else torch.float64
        out = torch.full((X.shape[0], e.n_features), float("nan"), dtype=dt, device="cuda")
        e.shap_values(X, precision, out=out)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        assert np.isfinite(got).all(), name
        check(got, oracle_mod.shap_values(wl.ensemble, wl.X, n=8), precision, name + " out=")


WIDE_CASES = [
    # Fashion-MNIST's width (784 features): full depth-8 random trees, 20%
    # integer columns, and grown deep trees (16/32 buckets) on 784 features
    ("c2_values", dict(F=784, T=24, M=150, n_train=20000)),
    ("c5_deep", dict(F=784, T=3, M=70, n_train=30000)),
]


@pytest.mark.parametrize("name,over", WIDE_CASES, ids=[c[0] for c in WIDE_CASES])
def test_wide_feature_space(q, oracle_mod, name, over):
    """784 features: the sample tile of all features does not fit in LDS, so
    each work item takes a segment of rows with at most 96 distinct features
    and stages only those.  Values and the adjoint, merged and plain tables,
    both precisions, with NaN rows, against the oracle."""
    print("case wide", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    ens = wl.ensemble
    X = wl.X.copy()
    rng = np.random.default_rng(7)
    X[rng.random(X.shape) < 0.03] = np.nan
    X[5] = np.nan
    assert ens.n_features == 784
    want = oracle_mod.shap_values(ens, X, n=8)
    G = rng.normal(size=(X.shape[0], ens.n_features))
    e = q.Ensemble(ens)
    Xd = torch.from_numpy(X).cuda()
    for merge in (True, False):
        e.set_sibling_merge(merge)
        for precision in ("fp32", "fp64"):
            got = e.shap_values(Xd, precision).double().cpu().numpy()
            err = check(got, want, precision, "wide %s merge=%s" % (name, merge))
            Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
            gw = oracle_mod.leaf_grad(ens, X, Gp)
            gl = e.shap_backward(Xd, torch.from_numpy(Gp).cuda(), precision).cpu().numpy()
            gerr = float(np.abs(gl - gw).max() / np.abs(gw).max())
            print("wide %s merge=%s %s: phi %.2e grad %.2e" % (name, merge, precision, err,
                                                              gerr), flush=True)
            assert gerr <= (1e-5 if precision == "fp32" else 1e-10)
