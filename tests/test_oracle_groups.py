"""Pins for the oracle's multi-output composition (a group of trees per
output): each output's game is the sum of its own trees' path-dependent games
(Eq. 3), so each output's Shapley values, interaction indices and leaf
gradients are those of its sub-ensemble.  Pinned by subset enumeration of each
output's game, by additivity over trees against the single-output oracle, by
copies of one ensemble in two outputs, by efficiency per output and by the
adjoint identity <grad_leaf, val> = <G, phi>."""
import numpy as np
import pytest

import synth
from oracle import brute


def _grouped(ens, K, seed=0):
    rng = np.random.default_rng(seed)
    tg = rng.integers(0, K, size=ens.n_trees)
    tg[:K] = np.arange(K)  # every output has a tree
    return ens.with_groups(tg, K, base_scores=rng.standard_normal(K))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_each_output_matches_enumeration(oracle_mod, seed):
    rng = np.random.default_rng(40 + seed)
    ens = synth.random_small_ensemble(rng, 7, 6, 4, zero_cover=(seed == 2))
    X = (np.round(rng.standard_normal((9, 6)) * 2) / 2).astype(np.float32)
    X[::3, 2] = np.nan
    g = _grouped(ens, 3, seed)
    phi = oracle_mod.shap_values_grouped(g, X)
    _, Phi = oracle_mod.shap_interactions_grouped(g, X)
    assert phi.shape == (9, 3, 6) and Phi.shape == (9, 3, 6, 6)
    for k in range(3):
        sub = ens.subset_trees(g.group_trees(k))
        np.testing.assert_allclose(phi[:, k], brute.shap_values(sub, X), rtol=0, atol=1e-12)
        sii = brute.shap_sii(sub, X)
        off = ~np.eye(6, dtype=bool)
        np.testing.assert_allclose(Phi[:, k][:, off], 0.5 * sii[:, off], rtol=0, atol=1e-12)


def test_outputs_add_up_to_the_single_output_model(oracle_mod):
    """Additivity over trees: the outputs' values sum to those of all trees
    as one output; one group reproduces the single-output oracle."""
    wl = synth.make_workload("c3_interactions", T=9, M=12, n_train=5000)
    ens, X = wl.ensemble, wl.X
    g = _grouped(ens, 4, 1)
    phi_all = oracle_mod.shap_values(ens, X)
    np.testing.assert_allclose(oracle_mod.shap_values_grouped(g, X).sum(1), phi_all,
                               rtol=0, atol=1e-12)
    p1, P1 = oracle_mod.shap_interactions_grouped(ens.with_groups(np.zeros(ens.n_trees), 1), X)
    p0, P0 = oracle_mod.shap_interactions(ens, X)
    np.testing.assert_allclose(p1[:, 0], p0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P1[:, 0], P0, rtol=0, atol=1e-15)
    _, Pg = oracle_mod.shap_interactions_grouped(g, X)
    np.testing.assert_allclose(Pg.sum(1), P0, rtol=0, atol=1e-12)


def test_copies_in_two_outputs(oracle_mod):
    wl = synth.make_workload("c1_small", M=20)
    ens = wl.ensemble
    twice = synth.ensembles._concat_trees(
        [{k: getattr(ens.subset_trees([t]), k) for k in ("left", "right", "feature",
                                                         "threshold", "default_left", "cover",
                                                         "value")}
         for t in list(range(ens.n_trees)) * 2], ens.n_features)
    g = twice.with_groups(np.repeat([0, 1], ens.n_trees), 2, base_scores=[0.25, -1.0])
    phi = oracle_mod.shap_values_grouped(g, wl.X)
    want = oracle_mod.shap_values(ens, wl.X)
    np.testing.assert_allclose(phi[:, 0], want, rtol=0, atol=1e-15)
    np.testing.assert_allclose(phi[:, 1], want, rtol=0, atol=1e-15)
    E = oracle_mod.expected_values_grouped(g)
    e0 = oracle_mod.expected_value(ens)
    np.testing.assert_allclose(E, [e0 + 0.25, e0 - 1.0], rtol=0, atol=1e-14)


def test_efficiency_per_output(oracle_mod):
    wl = synth.make_workload("c4_adjoint", T=12, M=30, n_train=5000, groups=3)
    g, X = wl.ensemble, wl.X
    assert g.n_groups == 3
    phi = oracle_mod.shap_values_grouped(g, X)
    fx = oracle_mod.predict_grouped(g, X)
    E = oracle_mod.expected_values_grouped(g)
    np.testing.assert_allclose(phi.sum(2) + E[None, :], fx, rtol=0, atol=1e-12)


def test_grouped_leaf_gradient(oracle_mod):
    """<grad_leaf, val> = <G, phi> (phi is linear in the leaf values), and
    the gradient of one output's G lands on that output's trees only."""
    wl = synth.make_workload("c4_adjoint", T=9, M=25, n_train=5000, groups=3)
    g, X = wl.ensemble, wl.X
    rng = np.random.default_rng(3)
    G = rng.standard_normal((X.shape[0], 3, g.n_features))
    grad = oracle_mod.leaf_grad_grouped(g, X, G)
    phi = oracle_mod.shap_values_grouped(g, X)
    vals = g.leaf_values()
    np.testing.assert_allclose(grad @ vals, np.sum(G * phi), rtol=1e-12)
    G1 = np.zeros_like(G)
    G1[:, 1] = G[:, 1]
    grad1 = oracle_mod.leaf_grad_grouped(g, X, G1)
    leaf_tree = np.repeat(np.arange(g.n_trees), [
        int((g.left[g.tree_offsets[t]:g.tree_offsets[t + 1]] < 0).sum())
        for t in range(g.n_trees)])
    assert np.all(grad1[g.tree_group[leaf_tree] != 1] == 0.0)
    assert np.abs(grad1[g.tree_group[leaf_tree] == 1]).max() > 0


def test_library_expected_values_and_group_validation(oracle_mod):
    import paper_2605_04497_amd as q
    wl = synth.make_workload("c2_values", T=7, M=4, n_train=5000, groups=3)
    e = q.Ensemble(wl.ensemble, host_only=True)
    assert e.n_groups == 3 and e.info["n_groups"] == 3
    np.testing.assert_allclose(e.expected_value, oracle_mod.expected_values_grouped(wl.ensemble),
                               rtol=0, atol=1e-12)
    bad = wl.ensemble.with_groups(np.full(wl.ensemble.n_trees, 3), 3)
    with pytest.raises(q.QtsError) as ei:
        q.Ensemble(bad, host_only=True)
    assert ei.value.code == -2
