"""GPU parity of the depth-first form of the pairwise interactions
(qts_set_pair_traversal 'dfs': section 5, Algorithm 1 at order 2 with the
telescoping update of Eq. 11) against the FP64 oracle's Phi and phi, in both
precisions: the workload shapes scaled down, irregular trees with repeated
features, zero covers and missing values, leaf-value overrides, chains of up
to 64 features, a triangle split into LDS ranges, output groups, graph
replay, several sample batches, and the full interactions ensemble."""
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


def _dfs(q, ens, X, precision, leaf_values=None, with_phi=True):
    e = q.Ensemble(ens)
    e.set_pair_traversal("dfs")
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    lv = None if leaf_values is None else torch.from_numpy(leaf_values).cuda()
    Phi, phi = e.shap_interactions(Xd, precision, leaf_values=lv, with_phi=True)
    torch.cuda.synchronize()
    return Phi.double().cpu().numpy(), phi.double().cpu().numpy(), e


CASES = [
    ("c1_small", dict(M=77)),
    ("c2_values", dict(T=12, M=41, n_train=20000)),       # integer ties
    ("c3_interactions", dict(T=6, M=37, n_train=20000)),  # depths 3..20
    ("c4_adjoint", dict(T=10, M=19, n_train=20000)),
    ("c5_deep", dict(T=3, M=21, n_train=30000)),          # depth 32, repeated features
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_dfs_matches_oracle(q, oracle_mod, name, over, precision):
    print("case dfs", name, over, precision, flush=True)
    wl = synth.make_workload(name, **over)
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X, n=8)
    Phi, phi, e = _dfs(q, wl.ensemble, wl.X, precision)
    assert e.info["n_dfs_nodes"] > 0
    err = check(Phi, Phi_o, precision, name + " dfs Phi")
    check(phi, phi_o, precision, name + " dfs phi")
    print("dfs %s %s: Phi %.2e" % (name, precision, err), flush=True)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dfs_irregular_trees(q, oracle_mod, seed):
    """Repeated features, ties, zero covers, NaN rows; a leaf-value override."""
    rng = np.random.default_rng(600 + seed)
    ens = synth.random_small_ensemble(rng, 7, 7, 7, n_train=300, zero_cover=(seed > 0))
    X = (np.round(rng.standard_normal((29, 7)) * 2) / 2).astype(np.float32)
    X[::3, ::2] = np.nan
    X[4] = np.nan
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        Phi, phi, _ = _dfs(q, ens, X, precision)
        check(Phi, Phi_o, precision, "irregular dfs")
        check(phi, phi_o, precision, "irregular dfs phi")
    lv = rng.standard_normal(ens.n_leaves())
    phi_o, Phi_o = oracle_mod.shap_interactions(ens.with_leaf_values(lv), X, n=8)
    Phi, phi, _ = _dfs(q, ens, X, "fp64", leaf_values=lv)
    check(Phi, Phi_o, "fp64", "override dfs")


def _chains(rng, n, F, D):
    trees = []
    for _ in range(n):
        feats = rng.permutation(F)[:D]
        b = rng.uniform(0.55, 0.95, D)
        cov = np.cumprod(np.concatenate([[1.0], b]))
        node = ("leaf", float(rng.standard_normal()), float(cov[D]))
        for j in reversed(range(D)):
            leaf = ("leaf", float(rng.standard_normal()), float(cov[j] * (1 - b[j])))
            thr = float(np.round(rng.standard_normal() * 0.8, 2))
            dl = int(rng.integers(2))
            node = (("split", int(feats[j]), thr, float(cov[j]), node, leaf, dl)
                    if rng.random() < 0.5 else
                    ("split", int(feats[j]), thr, float(cov[j]), leaf, node, dl))
        trees.append(node)
    return synth.from_nested(trees, n_features=F)


def test_dfs_chains_and_split_triangle(q, oracle_mod):
    """Chains of 64 distinct features (walk stacks 64 levels deep) and 300
    features, whose FP64 pair triangle takes several LDS ranges."""
    rng = np.random.default_rng(91)
    ens = _chains(rng, 3, 300, 64)
    X = (rng.standard_normal((5, 300)) * 0.6).astype(np.float32)
    X[2, ::9] = np.nan
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, X, n=8)
    for precision in ("fp32", "fp64"):
        Phi, phi, e = _dfs(q, ens, X, precision)
        assert e.info["max_depth"] == 64
        check(Phi, Phi_o, precision, "chains dfs")
        check(phi, phi_o, precision, "chains dfs phi")


def test_dfs_groups_and_replay(q, oracle_mod):
    wl = synth.make_workload("c3_interactions", T=9, M=23, n_train=20000, groups=3)
    ens = wl.ensemble
    pw, Pw = oracle_mod.shap_interactions_grouped(ens, wl.X)
    e = q.Ensemble(ens)
    e.set_pair_traversal("dfs")
    X = torch.from_numpy(wl.X).cuda()
    e.set_graph_replay(True)
    Phi = torch.empty((23, 3, 200, 200), device="cuda")
    phi = torch.empty((23, 3, 200), device="cuda")
    for _ in range(3):
        Phi.fill_(float("nan"))
        e.shap_interactions(X, "fp32", with_phi=True, out=Phi, out_phi=phi)
        torch.cuda.synchronize()
        check(Phi.double().cpu().numpy().reshape(69, -1), Pw.reshape(69, -1), "fp32",
              "grouped dfs replay")
        check(phi.double().cpu().numpy().reshape(69, -1), pw.reshape(69, -1), "fp32",
              "grouped dfs phi")
    e.set_graph_replay(False)


def test_dfs_full_interactions_ensemble_batches(q, oracle_mod):
    """The full 500-tree interactions ensemble on 1024 samples: the y values of
    one sample take 35 MB (FP32), so the call runs in several batches; rows
    checked at batch boundaries and spread over the samples."""
    wl = synth.make_workload("c3_interactions")
    M = 1024
    X = torch.from_numpy(wl.X[:M]).cuda()
    e = q.Ensemble(wl.ensemble)
    e.set_pair_traversal("dfs")
    rows = np.array([0, 119, 120, 511, 1023])
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X[rows], n=8)
    sel = torch.from_numpy(rows).cuda()
    for precision in ("fp32", "fp64"):
        Phi, phi = e.shap_interactions(X, precision, with_phi=True)
        torch.cuda.synchronize()
        err = check(Phi[sel].double().cpu().numpy(), Phi_o, precision, "c3 dfs Phi")
        check(phi[sel].double().cpu().numpy(), phi_o, precision, "c3 dfs phi")
        print("c3 dfs %s: %.2e" % (precision, err), flush=True)
        del Phi, phi
    e.close()


def test_dfs_edge_cases(q, oracle_mod):
    wl = synth.make_workload("c1_small", M=9)
    e = q.Ensemble(wl.ensemble)
    e.set_pair_traversal("dfs")
    F = e.n_features
    Phi = e.shap_interactions(torch.zeros((0, F), device="cuda"), "fp32")
    assert tuple(Phi.shape) == (0, F, F)
    X = torch.from_numpy(wl.X[:1]).cuda()
    _, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X[:1], n=8)
    check(e.shap_interactions(X, "fp64").cpu().numpy(), Phi_o, "fp64", "M = 1")
    # back to the path form on the same ensemble
    e.set_pair_traversal("paths")
    check(e.shap_interactions(X, "fp64").cpu().numpy(), Phi_o, "fp64", "paths again")
    # a tree that is a single leaf contributes nothing
    node = ("split", 1, 0.0, 1.0, ("leaf", 1.0, 0.5), ("leaf", -1.0, 0.5))
    e2 = q.Ensemble(synth.from_nested([("leaf", 3.0, 1.0), node], n_features=3))
    e2.set_pair_traversal("dfs")
    Xs = np.array([[0.5, -0.5, 1.0], [0.5, 0.5, np.nan]], np.float32)
    _, Phi_o = oracle_mod.shap_interactions(
        synth.from_nested([("leaf", 3.0, 1.0), node], n_features=3), Xs, n=8)
    check(e2.shap_interactions(torch.from_numpy(Xs).cuda(), "fp64").cpu().numpy(), Phi_o,
          "fp64", "single-leaf tree")


def test_auto_traversal_keeps_parity(q, oracle_mod):
    """'auto': the autotuner times both forms and keeps the faster per
    precision; whichever it keeps matches the oracle."""
    wl = synth.make_workload("c5_deep", T=6, M=64, n_train=30000)
    e = q.Ensemble(wl.ensemble)
    e.set_pair_traversal("auto")
    assert e.info["pairs_dfs"] == 0          # the path form until tuned
    X = torch.from_numpy(wl.X).cuda()
    _, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X, n=8)
    for precision in ("fp32", "fp64"):
        e.autotune(64, precision)
        info = e.refresh_info()
        print("auto traversal %s: pairs_dfs=%d" % (precision, info["pairs_dfs"]), flush=True)
        check(e.shap_interactions(X, precision).double().cpu().numpy(), Phi_o, precision,
              "auto traversal")
