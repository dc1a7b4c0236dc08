"""GPU parity of qts_shap_interactions (Phi[M,F,F], and phi) against the FP64
oracle's 8-node pair indices, with the convention Phi_ik = SII_ik / 2 (i != k)
and Phi_ii = phi_i - sum_{k != i} Phi_ik."""
import functools

import numpy as np
import pytest

import synth
from tests.parity import check, row_normwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def q():
    import paper_2605_04497_amd as q
    return q


def _run(q, ens, X, precision, leaf_values=None):
    e = q.Ensemble(ens)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lv = None if leaf_values is None else torch.from_numpy(leaf_values).cuda()
    Phi, phi = e.shap_interactions(Xd, precision, leaf_values=lv, with_phi=True)
    torch.cuda.synchronize()
    return Phi.cpu().numpy().astype(np.float64), phi.cpu().numpy().astype(np.float64), e


CASES = [
    ("c1_small", dict(M=70)),
    ("c3_interactions", dict(T=4, M=20, n_train=20000)),   # F=200, depths 3..20
    ("c4_adjoint", dict(T=10, M=70, n_train=20000)),
    ("c5_deep", dict(T=3, M=12, n_train=30000)),           # long paths: lane groups
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_interactions_match_oracle(q, oracle_mod, name, over, precision):
    print("case", name, over, precision, flush=True)
    wl = synth.make_workload(name, **over)
    Phi, phi, e = _run(q, wl.ensemble, wl.X, precision)
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X, n=8)
    check(Phi, Phi_o, precision, name + " Phi")
    check(phi, phi_o, precision, name + " phi")
    np.testing.assert_array_equal(Phi, np.transpose(Phi, (0, 2, 1)))  # symmetric by construction
    tol = 1e-5 if precision == "fp32" else 1e-10
    scale = np.maximum(np.abs(phi_o).max(1, keepdims=True), 1e-30)
    assert np.all(np.abs(Phi.sum(2) - phi) <= tol * scale)            # rows sum to phi


def test_c1_pairs_match_enumeration(q):
    """Pair indices from the GPU vs subset enumeration of the Shapley
    interaction index definition (F = 8, exact at d <= 4)."""
    from oracle import brute
    wl = synth.make_workload("c1_small", M=10)
    Phi, phi, _ = _run(q, wl.ensemble, wl.X, "fp64")
    sii = brute.shap_sii(wl.ensemble, wl.X)
    off = ~np.eye(wl.ensemble.n_features, dtype=bool)
    assert row_normwise(2 * Phi * off, sii) <= 1e-10
    assert row_normwise(phi, brute.shap_values(wl.ensemble, wl.X)) <= 1e-10


def test_interactions_phi_matches_values_kernel(q):
    wl = synth.make_workload("c2_values", T=20, M=100, n_train=20000)
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    for precision in ("fp32", "fp64"):
        _, phi = e.shap_interactions(X, precision, with_phi=True)
        phi2 = e.shap_values(X, precision)
        assert row_normwise(phi.double().cpu().numpy(), phi2.double().cpu().numpy()) <= (
            2e-6 if precision == "fp32" else 1e-12)


def test_interactions_edge_cases(q, oracle_mod):
    # zero covers (paths whose factor vanishes), repeated features, NaN rows
    for seed in range(3):
        rng = np.random.default_rng(400 + seed)
        ens = synth.random_small_ensemble(rng, 5, 9, 7, zero_cover=True)
        X = (np.round(rng.standard_normal((67, 9)) * 2) / 2).astype(np.float32)
        X[::5, 3] = np.nan
        X[7, :] = np.nan
        phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
        for precision in ("fp32", "fp64"):
            Phi, phi, _ = _run(q, ens, X, precision)
            check(Phi, Phi_o, precision, "zero covers Phi")
            check(phi, phi_o, precision, "zero covers phi")
    # leaf-value override, M = 1 and M = 0
    wl = synth.make_workload("c4_adjoint", T=4, M=9, n_train=5000)
    v = np.random.default_rng(2).normal(size=wl.ensemble.n_leaves())
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble.with_leaf_values(v), wl.X)
    for precision in ("fp32", "fp64"):
        Phi, _, _ = _run(q, wl.ensemble, wl.X, precision, leaf_values=v)
        check(Phi, Phi_o, precision, "leaf override")
        Phi1, _, _ = _run(q, wl.ensemble, wl.X[4:5], precision, leaf_values=v)
        check(Phi1, Phi_o[4:5], precision, "M=1")
    e = q.Ensemble(wl.ensemble)
    out = e.shap_interactions(torch.zeros((0, wl.ensemble.n_features), device="cuda"))
    assert out.shape == (0, wl.ensemble.n_features, wl.ensemble.n_features)


@pytest.mark.parametrize("d", [3, 12, 13, 20, 21, 24, 25, 28, 29, 32, 33, 36, 37, 40, 41, 48, 64])
def test_interaction_capacity_classes(q, oracle_mod, d):
    """A chain of d features covers each capacity class boundary: the one-lane
    classes, the classes whose paths take two or four lanes (FP32 24..40,
    FP64 24..28) and the long-path (generic) classes."""
    from tests.test_gpu_values import chain_model, chain_rows
    ens, X = chain_model(d), chain_rows(d)
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        Phi, phi, _ = _run(q, ens, X, precision)
        check(Phi, Phi_o, precision, "chain d=%d" % d)


@pytest.mark.parametrize("F", [202, 300])
def test_interactions_split_triangle(q, oracle_mod, F):
    """More features than one FP64 pair triangle fits in LDS: the triangle is
    cut into row ranges, one launch each; every range must add its pairs once
    and phi must be added by the first range only."""
    rng = np.random.default_rng(600 + F)
    ens = synth.random_small_ensemble(rng, 12, F, 9)
    X = rng.standard_normal((37, F)).astype(np.float32)
    X[::4, ::7] = np.nan
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        Phi, phi, _ = _run(q, ens, X, precision)
        check(Phi, Phi_o, precision, "F=%d Phi" % F)
        check(phi, phi_o, precision, "F=%d phi" % F)


def test_merged_sibling_rows_cancellation(q, oracle_mod):
    """Rows that merge two sibling leaves carry a combined factor that can
    vanish at a node (equal and opposite leaf values, zero covers); pairs and
    phi must still match the oracle, via the model's values and an override."""
    from tests.test_gpu_values import _sibling_leaf_pairs
    for seed in range(3):
        rng = np.random.default_rng(800 + seed)
        ens = synth.random_small_ensemble(rng, 8, 9, 7, zero_cover=(seed == 1))
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
        X = (np.round(rng.standard_normal((61, 9)) * 2) / 2).astype(np.float32)
        X[::4, 2] = np.nan
        phi_o, Phi_o = oracle_mod.shap_interactions(ens.with_leaf_values(v), X, n=8)
        for precision in ("fp32", "fp64"):
            Phi, phi, _ = _run(q, ens.with_leaf_values(v), X, precision)
            check(Phi, Phi_o, precision, "sibling values Phi")
            check(phi, phi_o, precision, "sibling values phi")
            Phi, phi, _ = _run(q, ens, X, precision, leaf_values=v)
            check(Phi, Phi_o, precision, "override Phi")


def test_long_paths_with_split_triangle(q, oracle_mod):
    """Paths of more than 24 features (two or four lanes per path) together
    with more features than one LDS triangle holds (row ranges), in both
    precisions."""
    rng = np.random.default_rng(900)
    ens = synth.random_small_ensemble(rng, 3, 260, 34, n_train=4000, p_leaf=0.0)
    X = rng.standard_normal((23, 260)).astype(np.float32)
    X[::6, ::11] = np.nan
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        Phi, phi, e = _run(q, ens, X, precision)
        assert e.info["max_unique"] > 24
        check(Phi, Phi_o, precision, "long paths Phi")
        check(phi, phi_o, precision, "long paths phi")


@pytest.mark.parametrize("name,over", [
    ("c1_small", dict(M=40)),                                  # classes 4 and 8
    ("c3_interactions", dict(T=6, M=24, n_train=20000)),       # classes 4..20
])
def test_interactions_exact_node_policy(q, oracle_mod, name, over):
    """With the 'exact' node policy, capacity classes 4, 8 and 12 use the
    2-, 4- and 6-node rules; their pair integrands have degree <= C - 2 (and
    first-order ones <= C - 1), so Phi and phi equal the 8-node oracle's up to
    rounding.  Longer classes keep 8 nodes."""
    print("case", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    e.set_node_policy("exact")
    X = torch.from_numpy(wl.X).cuda()
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X, n=8)
    for precision in ("fp32", "fp64"):
        dt = torch.float32 if precision == "fp32" else torch.float64
        Phi = torch.empty((X.shape[0], e.n_features, e.n_features), dtype=dt, device="cuda")
        phi = torch.empty((X.shape[0], e.n_features), dtype=dt, device="cuda")
        e.shap_interactions(X, precision, with_phi=True, out=Phi, out_phi=phi)
        torch.cuda.synchronize()
        check(Phi.double().cpu().numpy(), Phi_o, precision, name + " exact Phi")
        check(phi.double().cpu().numpy(), phi_o, precision, name + " exact phi")


def _random_chains(rng, n_chains, F, D):
    """Chains of D distinct features drawn from F: at each split a random side
    continues and the other is a leaf, with random thresholds, missing-value
    directions and cover ratios, so the rows of one chain have 1..D unique
    features and fill every capacity class up to D."""
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


def test_every_class_with_many_rows(q, oracle_mod):
    """Several rows in every capacity class from 4 to 64: one-lane instances
    with node passes, two- and four-lane groups (ragged in the last group of
    a wave) and the wave-per-path kernel, over a triangle split into row
    ranges (F = 260), with missing values, in both precisions."""
    rng = np.random.default_rng(4242)
    ens = _random_chains(rng, 5, 260, 64)
    X = rng.standard_normal((29, 260)).astype(np.float32) * 0.6
    X[::5, ::9] = np.nan
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        Phi, phi, e = _run(q, ens, X, precision)
        assert e.info["max_unique"] == 64
        check(Phi, Phi_o, precision, "chains Phi")
        check(phi, phi_o, precision, "chains phi")
