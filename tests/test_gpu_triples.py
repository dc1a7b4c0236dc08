"""GPU parity of the third-order Shapley interaction indices
(qts_shap_interactions3: Theorem 1 with |S| = 3, Eq. 9-10) against the FP64
oracle's dense [M, F, F, F] tensor, in both precisions: merged sibling rows
(short ones in the lane-per-row kernel, rows of 9 to 16 features in the
wave-per-row kernel), missing values, every capacity class up to 64 slots, a
tensor split into ranges of its largest feature, leaf-value overrides and the
empty cases."""
import numpy as np
import pytest

import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def q():
    import paper_2605_04497_amd as q
    return q


def packed(dense):
    """[M, F, F, F] -> [M, F(F-1)(F-2)/6], triple i < j < k at k(k-1)(k-2)/6 + j(j-1)/2 + i."""
    F = dense.shape[1]
    out = np.zeros((dense.shape[0], F * (F - 1) * (F - 2) // 6))
    for k in range(F):
        for j in range(k):
            for i in range(j):
                out[:, k * (k - 1) * (k - 2) // 6 + j * (j - 1) // 2 + i] = dense[:, i, j, k]
    return out


def _run(q, ens, X, precision, leaf_values=None):
    e = q.Ensemble(ens)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lv = None if leaf_values is None else torch.from_numpy(leaf_values).cuda()
    out = e.shap_interactions3(Xd, precision, leaf_values=lv)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), e


def _chains(rng, n_chains, F, D):
    """Random chains of D distinct features (a random side continues at every
    split), so each chain's rows have 1..D unique features."""
    trees = []
    for _ in range(n_chains):
        feats = rng.permutation(F)[:D]
        b = rng.uniform(0.55, 0.95, D)
        cov = np.cumprod(np.concatenate([[1.0], b]))
        node = ("leaf", float(rng.standard_normal()), float(cov[D]))
        for j in reversed(range(D)):
            leaf = ("leaf", float(rng.standard_normal()), float(cov[j] * (1 - b[j])))
            thr = float(np.round(rng.standard_normal() * 0.8, 2))
            dl = int(rng.integers(2))
            if rng.random() < 0.5:
                node = ("split", int(feats[j]), thr, float(cov[j]), node, leaf, dl)
            else:
                node = ("split", int(feats[j]), thr, float(cov[j]), leaf, node, dl)
        trees.append(node)
    return synth.from_nested(trees, n_features=F)


@pytest.mark.parametrize("name,over", [
    ("c1_small", dict(M=30)),
    ("c4_adjoint", dict(T=4, M=9, n_train=20000, F=12)),
])
def test_triples_match_oracle(q, oracle_mod, name, over):
    """Workload ensembles at small sizes (merged sibling rows, full trees)."""
    print("case", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    want = packed(oracle_mod.shap_sii3(wl.ensemble, wl.X, n=8))
    assert np.abs(want).max() > 0
    for precision in ("fp32", "fp64"):
        got, e = _run(q, wl.ensemble, wl.X, precision)
        check(got, want, precision, name)


@pytest.mark.parametrize("seed", [0, 1])
def test_triples_irregular_trees_missing_values(q, oracle_mod, seed):
    """Small irregular trees with repeated features, ties, zero covers and
    missing values; one leaf-value override."""
    rng = np.random.default_rng(300 + seed)
    ens = synth.random_small_ensemble(rng, 6, 9, 6, n_train=400, zero_cover=(seed == 1))
    X = (np.round(rng.standard_normal((21, 9)) * 2) / 2).astype(np.float32)
    X[::4, ::3] = np.nan
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    for precision in ("fp32", "fp64"):
        got, e = _run(q, ens, X, precision)
        check(got, want, precision, "irregular seed %d" % seed)
    lv = rng.standard_normal(ens.n_leaves())
    want = packed(oracle_mod.shap_sii3(ens.with_leaf_values(lv), X, n=8))
    got, e = _run(q, ens, X, "fp64", leaf_values=lv)
    check(got, want, "fp64", "leaf override")


def test_triples_long_rows_and_split_tensor(q, oracle_mod):
    """Chains of 40 features out of 70 (rows in every class up to 40 slots)
    and a packed tensor of 54,740 triples, more than one LDS range holds."""
    rng = np.random.default_rng(77)
    ens = _chains(rng, 3, 70, 40)
    X = (rng.standard_normal((3, 70)) * 0.6).astype(np.float32)
    X[1, ::5] = np.nan
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    for precision in ("fp32", "fp64"):
        got, e = _run(q, ens, X, precision)
        assert e.info["max_unique"] == 40
        check(got, want, precision, "chains")


def test_triples_dense_expansion_and_empty_cases(q, oracle_mod):
    wl = synth.make_workload("c1_small", M=5)
    dense = oracle_mod.shap_sii3(wl.ensemble, wl.X, n=8)
    got, e = _run(q, wl.ensemble, wl.X, "fp64")
    full = e.triples_dense(torch.from_numpy(got), e.n_features).numpy()
    check(full, dense, "fp64", "dense expansion")
    # no samples
    out = e.shap_interactions3(torch.zeros((0, e.n_features), device="cuda"), "fp32")
    assert tuple(out.shape) == (0, e.n_features * (e.n_features - 1) * (e.n_features - 2) // 6)
    # fewer than three features: nothing to compute
    node = ("split", 1, 0.0, 1.0, ("leaf", 1.0, 0.5), ("leaf", -1.0, 0.5))
    e2 = q.Ensemble(synth.from_nested([node], n_features=2))
    out = e2.shap_interactions3(torch.zeros((4, 2), device="cuda"), "fp64")
    assert tuple(out.shape) == (4, 0)


def test_triples_deep_grown_merged_rows(q, oracle_mod):
    """A few grown depth-32 trees (the deep workload's structure): rows of up
    to ~30 features, including merged sibling rows of 9 to 16 features, which
    take the merged branch of the wave-per-row kernel in classes 12 and 16."""
    wl = synth.make_workload("c5_deep", T=3, M=4, n_train=30000)
    e0 = q.Ensemble(wl.ensemble)
    assert e0.info["max_unique"] > 16
    pt_rows = e0.info["n_pair_rows"]
    assert pt_rows < e0.info["n_paths"]  # some rows are merged sibling pairs
    want = packed(oracle_mod.shap_sii3(wl.ensemble, wl.X, n=8))
    assert np.abs(want).max() > 0
    for precision in ("fp32", "fp64"):
        got, e = _run(q, wl.ensemble, wl.X, precision)
        err = check(got, want, precision, "deep grown")
        print("deep grown triples %s: %.2e" % (precision, err), flush=True)


def test_triples_chains_of_64(q, oracle_mod):
    """Chains of 64 distinct features out of 72: rows in the 48- and 64-slot
    classes (the longest instances), a tensor of 59,640 triples cut into
    several LDS ranges, missing values on one sample."""
    rng = np.random.default_rng(78)
    ens = _chains(rng, 2, 72, 64)
    X = (rng.standard_normal((2, 72)) * 0.6).astype(np.float32)
    X[1, ::7] = np.nan
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    for precision in ("fp32", "fp64"):
        got, e = _run(q, ens, X, precision)
        assert e.info["max_unique"] == 64
        err = check(got, want, precision, "chains of 64")
        print("chains of 64 triples %s: %.2e" % (precision, err), flush=True)
