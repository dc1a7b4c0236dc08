"""GPU parity of the depth-first form of the third-order interaction indices
(qts_shap_interactions3 under qts_set_pair_traversal 'dfs': Algorithm 1 of
section 5 taken to order 3, Theorem 1 with |S| = 3) against the FP64
oracle's dense [M, F, F, F] tensor, in both precisions: the workload shapes
scaled down, irregular trees with repeated features, zero covers and missing
values, leaf-value overrides, rows of up to 31 features, a tensor cut into
LDS ranges, output groups, the autotuner's choice, the fall-back to the path
form for rows longer than the pass holds, and several sample batches."""
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
    F = dense.shape[-1]
    out = np.zeros(dense.shape[:-3] + (F * (F - 1) * (F - 2) // 6,))
    for c in range(F):
        for b in range(c):
            for a in range(b):
                out[..., c * (c - 1) * (c - 2) // 6 + b * (b - 1) // 2 + a] = dense[..., a, b, c]
    return out


def _run(q, ens, X, precision, leaf_values=None, traversal="dfs"):
    e = q.Ensemble(ens)
    e.set_pair_traversal(traversal)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lv = None if leaf_values is None else torch.from_numpy(leaf_values).cuda()
    out = e.shap_interactions3(Xd, precision, leaf_values=lv)
    torch.cuda.synchronize()
    return out.double().cpu().numpy(), e


def _chains(rng, n_chains, F, D):
    """Chains of D distinct features (a random side continues at every split)."""
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


CASES = [
    ("c1_small", dict(M=30)),
    ("c3_interactions", dict(T=4, M=5, n_train=20000, F=40)),  # depths 3..20
    ("c4_adjoint", dict(T=6, M=9, n_train=20000, F=12)),
    ("c5_deep", dict(T=3, M=4, n_train=30000)),                # depth 32, repeated features
]


@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_dfs3_matches_oracle(q, oracle_mod, name, over):
    print("case dfs3", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    want = packed(oracle_mod.shap_sii3(wl.ensemble, wl.X, n=8))
    assert np.abs(want).max() > 0
    for precision in ("fp32", "fp64"):
        got, e = _run(q, wl.ensemble, wl.X, precision)
        assert e.info["pairs_dfs"] & (4 if precision == "fp32" else 8)
        assert e.info["n_dfs_updates3"] > 0
        err = check(got, want, precision, name + " dfs3")
        print("dfs3 %s %s: %.2e" % (name, precision, err), flush=True)


@pytest.mark.parametrize("seed", [0, 1])
def test_dfs3_irregular_trees_missing_values(q, oracle_mod, seed):
    """Repeated features, ties, zero covers, NaN rows; a leaf-value override."""
    rng = np.random.default_rng(700 + seed)
    ens = synth.random_small_ensemble(rng, 6, 9, 6, n_train=400, zero_cover=(seed == 1))
    X = (np.round(rng.standard_normal((21, 9)) * 2) / 2).astype(np.float32)
    X[::4, ::3] = np.nan
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    for precision in ("fp32", "fp64"):
        got, e = _run(q, ens, X, precision)
        check(got, want, precision, "dfs3 irregular seed %d" % seed)
    lv = rng.standard_normal(ens.n_leaves())
    want = packed(oracle_mod.shap_sii3(ens.with_leaf_values(lv), X, n=8))
    got, e = _run(q, ens, X, "fp64", leaf_values=lv)
    check(got, want, "fp64", "dfs3 leaf override")


def test_dfs3_long_rows_split_tensor_and_fallback(q, oracle_mod):
    """Chains of 31 features out of 70 (rows of up to 30 features above a
    node: the 32-slot pass; a tensor of 54,740 triples cut into LDS ranges),
    and chains of 40, whose rows the pass cannot hold: 'dfs' then keeps the
    path form for third order, with the same results."""
    rng = np.random.default_rng(79)
    ens = _chains(rng, 3, 70, 31)
    X = (rng.standard_normal((3, 70)) * 0.6).astype(np.float32)
    X[1, ::5] = np.nan
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    for precision in ("fp32", "fp64"):
        got, e = _run(q, ens, X, precision)
        assert e.info["pairs_dfs"] & (4 if precision == "fp32" else 8)
        check(got, want, precision, "dfs3 chains of 31")
    ens = _chains(rng, 2, 50, 40)
    X = (rng.standard_normal((2, 50)) * 0.6).astype(np.float32)
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    got, e = _run(q, ens, X, "fp64")
    assert e.info["pairs_dfs"] & 8 == 0
    check(got, want, "fp64", "chains of 40: path form")


def test_dfs3_groups(q, oracle_mod):
    wl = synth.make_workload("c4_adjoint", T=9, M=7, n_train=20000, F=12, groups=3)
    ens, X = wl.ensemble, wl.X
    want3 = oracle_mod.shap_sii3_grouped(ens, X)
    for precision in ("fp32", "fp64"):
        got, e = _run(q, ens, X, precision)
        assert got.shape == (7, 3, 12 * 11 * 10 // 6)
        check(got.reshape(21, -1), packed(want3).reshape(21, -1), precision, "dfs3 groups")


def test_dfs3_auto_choice(q, oracle_mod):
    """'auto': the autotuner times both third-order forms; whichever it keeps
    matches the oracle."""
    wl = synth.make_workload("c5_deep", T=4, M=6, n_train=30000)
    e = q.Ensemble(wl.ensemble)
    assert e.info["pairs_dfs"] == 0
    X = torch.from_numpy(wl.X).cuda()
    want = packed(oracle_mod.shap_sii3(wl.ensemble, wl.X, n=8))
    for precision in ("fp32", "fp64"):
        e.autotune(6, precision)
        print("auto dfs3 %s: pairs_dfs=%d" % (precision, e.refresh_info()["pairs_dfs"]),
              flush=True)
        check(e.shap_interactions3(X, precision).double().cpu().numpy(), want, precision,
              "dfs3 auto")


def test_dfs3_batches_agree(q):
    """The full interactions ensemble (1.1M internal nodes) takes the samples
    in batches whose y values fit the walk's scratch: 130 samples in several
    batches give the same tensors as the last five alone (one batch).  F = 200
    is beyond the path form's third-order kernels: only this form serves it."""
    wl = synth.make_workload("c3_interactions", M=130)
    e = q.Ensemble(wl.ensemble)
    e.set_pair_traversal("dfs")
    X = torch.from_numpy(wl.X).cuda()
    full = e.shap_interactions3(X, "fp64")
    tail = e.shap_interactions3(X[125:].contiguous(), "fp64")
    torch.cuda.synchronize()
    a = full[125:].cpu().numpy()
    b = tail.cpu().numpy()
    assert np.abs(b).max() > 0
    err = float(np.abs(a - b).max() / np.abs(b).max())
    print("dfs3 batches: max rel diff %.2e" % err, flush=True)
    assert err <= 1e-12


def test_dfs3_auto_wide_features(q, oracle_mod):
    """F = 240, beyond what the path form's third-order kernels hold in LDS
    (one feature's triples fit up to F = 203 for rows of at most 8 features).
    Under 'auto' an untuned ensemble takes the path form and reports
    QTS_E_UNSUPPORTED (a host-side check, before any third-order kernel);
    after qts_autotune it takes the depth-first form, which matches the
    oracle in both precisions."""
    from paper_2605_04497_amd import _lib as L
    rng = np.random.default_rng(23)
    F = 240
    ens = _chains(rng, 3, F, 6)
    X = rng.standard_normal((3, F)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    e = q.Ensemble(ens)
    with pytest.raises(L.QtsError) as ei:
        e.shap_interactions3(Xd, "fp32")
        torch.cuda.synchronize()
    assert ei.value.code == L.QTS_E_UNSUPPORTED
    want = packed(oracle_mod.shap_sii3(ens, X, n=8))
    assert np.abs(want).max() > 0
    for precision in ("fp32", "fp64"):
        e.autotune(3, precision)
        got = e.shap_interactions3(Xd, precision)
        torch.cuda.synchronize()
        check(got.double().cpu().numpy(), want, precision, "dfs3 auto, F = 240")
