"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics,
not by the oracle itself: hand-derived closed forms (golden files), subset
enumeration from the Shapley / interaction definitions, recursive TreeSHAP,
Gauss-Legendre exactness, and the invariants of Shapley values."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- quadrature
def _mp_rule(n):
    """n-point Gauss-Legendre rule on [0,1] in 40-digit arithmetic (mpmath):
    roots of P_n refined from numpy's, weights 2/((1-x^2) P_n'(x)^2) / 2."""
    import mpmath as mp
    mp.mp.dps = 40
    x0, _ = np.polynomial.legendre.leggauss(n)
    t, w = [], []
    for r in sorted(x0):
        x = mp.findroot(lambda z: mp.legendre(n, z), mp.mpf(r))
        dp = mp.diff(lambda z: mp.legendre(n, z), x)
        t.append((1 + x) / 2)
        w.append(1 / ((1 - x * x) * dp * dp))
    return t, w


def test_gauss_legendre_matches_high_precision_and_is_exact(oracle_mod):
    """The rule on [0,1] (Eq. 10): nodes and weights equal a 40-digit
    computation to rounding, agree with numpy's rule, and integrate t^k
    exactly for k <= 2n-1 (Theorem 2)."""
    for n in (1, 2, 3, 5, 8, 13, 32):
        t, s, w = oracle_mod.gauss_legendre(n)
        tm, wm = _mp_rule(n)
        np.testing.assert_allclose(t, [float(v) for v in tm], rtol=0, atol=2e-16)
        np.testing.assert_allclose(s, [float(1 - v) for v in tm], rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, [float(v) for v in wm], rtol=1e-14, atol=0)
        x, W = np.polynomial.legendre.leggauss(n)
        order = np.argsort((1 + x) / 2)
        np.testing.assert_allclose(w, (W / 2)[order], rtol=2e-13, atol=0)
        for k in range(2 * n):
            np.testing.assert_allclose(np.sum(w * t ** k), 1.0 / (k + 1), rtol=1e-14)
        if n <= 8:  # degree 2n is not integrated exactly
            assert abs(np.sum(w * t ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-15


# ---------------------------------------------------------------- closed forms
def test_stump_closed_form(oracle_mod):
    g = _gold("stump.json")
    m = g["model"]
    ens = synth.stump(m["n_left"], m["n_right"], m["v_left"], m["v_right"], m["threshold"])
    X = np.array(g["X"], np.float32)
    assert oracle_mod.expected_value(ens) == pytest.approx(g["expected_value"], abs=1e-15)
    np.testing.assert_allclose(oracle_mod.predict(ens, X), g["prediction"], atol=0)
    for n in (1, 8, 32):
        np.testing.assert_allclose(oracle_mod.shap_values(ens, X, n=n), g["phi"], atol=1e-15)
    np.testing.assert_allclose(oracle_mod.treeshap(ens, X), g["phi"], atol=1e-15)
    np.testing.assert_allclose(brute.shap_values(ens, X), g["phi"], atol=1e-15)


def _two_player():
    return synth.from_nested([
        ("split", 0, 0.0, 100.0,
         ("split", 1, 0.0, 40.0, ("leaf", 4.0, 10.0), ("leaf", -2.0, 30.0)),
         ("leaf", 1.0, 60.0))], n_features=2)


def test_two_player_closed_form(oracle_mod):
    g = _gold("two_player.json")
    ens = _two_player()
    x = np.array([g["x"]], np.float32)
    for key, val in g["game"].items():
        assert brute.game_value(ens, x[0], {int(c) for c in key}) == pytest.approx(val, abs=1e-15)
    assert oracle_mod.expected_value(ens) == pytest.approx(g["expected_value"], abs=1e-15)
    assert oracle_mod.predict(ens, x)[0] == pytest.approx(g["prediction"], abs=1e-15)
    for n in (1, 8, 32):  # d = 2: one node already integrates degree 1 exactly
        phi, Phi = oracle_mod.shap_interactions(ens, x, n=n)
        np.testing.assert_allclose(phi[0], g["phi"], atol=1e-14)
        np.testing.assert_allclose(Phi[0], g["Phi"], atol=1e-14)
    _, sii = oracle_mod.shap_sii(ens, x)
    assert sii[0, 0, 1] == pytest.approx(g["sii_01"], abs=1e-14)
    assert sii[0, 1, 0] == pytest.approx(g["sii_01"], abs=1e-14)
    np.testing.assert_allclose(oracle_mod.treeshap(ens, x)[0], g["phi"], atol=1e-14)


def _chain(d, b, val, F=None):
    """Feature j splits at depth j; x follows the left branch, whose cover
    ratio is b; every right branch is a leaf of value 0; the deepest left leaf
    has value `val`.  Only one path carries value: every b_j = b, o_j = 1."""
    F = F or d
    cov = 1.0
    node = ("leaf", val, b ** d)
    for j in reversed(range(d)):
        cov = b ** j
        node = ("split", j, 0.0, cov, node, ("leaf", 0.0, cov * (1 - b)))
    return synth.from_nested([node], n_features=F)


@pytest.mark.parametrize("d,b", [(1, 0.3), (4, 0.5), (9, 0.25), (16, 0.5), (17, 0.5),
                                 (32, 0.5), (32, 0.1), (48, 0.9)])
def test_single_followed_path_closed_form(oracle_mod, d, b):
    """phi_i = val * (1-b^d) / d for every feature on a followed path with all
    b_j = b: the integral of val*(1-b)*(b+(1-b)t)^(d-1) over [0,1]."""
    val = 1.5
    ens = _chain(d, b, val, F=d + 2)
    x = np.full((1, d + 2), -1.0, np.float32)
    want = val * (1 - b ** d) / d
    phi32 = oracle_mod.shap_values(ens, x, n=32)[0]
    np.testing.assert_allclose(phi32[:d], want, rtol=1e-13)
    assert np.all(phi32[d:] == 0.0)  # null players: exactly zero
    phi8 = oracle_mod.shap_values(ens, x, n=8)[0]
    if d <= 16:  # degree d-1 <= 15 = 2*8-1: the 8-node rule is exact
        np.testing.assert_allclose(phi8[:d], want, rtol=1e-13)
    else:
        rel = np.max(np.abs(phi8[:d] - want)) / abs(want)
        assert rel < 5e-3  # truncation only, shrinking as b -> 1
    if d <= 32:
        np.testing.assert_allclose(oracle_mod.treeshap(ens, x)[0][:d], want, rtol=1e-10)


# ---------------------------------------------------------------- enumeration
@pytest.mark.parametrize("seed", range(6))
def test_quadrature_equals_enumeration_and_treeshap(oracle_mod, seed):
    """Subset enumeration of the Shapley value / pair index definitions, the
    exact path quadrature, the 8-node rule (exact for d <= 16) and recursive
    TreeSHAP agree on small irregular trees with repeated features, ties and
    missing values."""
    rng = np.random.default_rng(100 + seed)
    ens = synth.random_small_ensemble(rng, 3, 6, 5)
    X = (np.round(rng.standard_normal((5, 6)) * 2) / 2).astype(np.float32)
    X[0, rng.integers(6)] = np.nan
    X[1, :] = np.nan
    phi_b = brute.shap_values(ens, X)
    sii_b = brute.shap_sii(ens, X)
    scale = max(1.0, np.abs(phi_b).max())
    for n in (8, 32):
        phi_q, sii_q = oracle_mod.shap_sii(ens, X, n=n)
        np.testing.assert_allclose(phi_q, phi_b, atol=1e-13 * scale)
        np.testing.assert_allclose(sii_q, sii_b, atol=1e-13 * scale)
    np.testing.assert_allclose(oracle_mod.treeshap(ens, X), phi_b, atol=1e-12 * scale)


def test_enumeration_over_all_players_matches_per_tree():
    """Null players do not change Shapley values: enumerating every feature of
    [F] gives the same phi as enumerating each tree's own features."""
    rng = np.random.default_rng(7)
    ens = synth.random_small_ensemble(rng, 2, 5, 3)
    X = rng.standard_normal((3, 5)).astype(np.float32)
    from math import factorial
    import itertools
    F = ens.n_features
    for r in range(X.shape[0]):
        want = brute.shap_values(ens, X[r:r + 1])[0]
        for i in range(F):
            rest = [f for f in range(F) if f != i]
            tot = 0.0
            for k in range(F):
                wgt = factorial(k) * factorial(F - k - 1) / factorial(F)
                for T in itertools.combinations(rest, k):
                    tot += wgt * (brute.game_value(ens, X[r], set(T) | {i})
                                  - brute.game_value(ens, X[r], set(T)))
            assert tot == pytest.approx(want[i], abs=1e-13)


def test_zero_cover_game(oracle_mod):
    """Zero parent covers give w_e = 0 (a valid game); quadrature still equals
    enumeration of the definition."""
    for seed in range(4):
        rng = np.random.default_rng(200 + seed)
        ens = synth.random_small_ensemble(rng, 3, 5, 4, zero_cover=True)
        assert (ens.cover == 0).any() or seed > 0
        X = (np.round(rng.standard_normal((4, 5)) * 2) / 2).astype(np.float32)
        phi_b = brute.shap_values(ens, X)
        sii_b = brute.shap_sii(ens, X)
        phi_q, sii_q = oracle_mod.shap_sii(ens, X, n=32)
        np.testing.assert_allclose(phi_q, phi_b, atol=1e-13)
        np.testing.assert_allclose(sii_q, sii_b, atol=1e-13)


# ---------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def mid_workload():
    w = synth.make_workload("c5_deep", T=6, M=12, n_train=20_000)
    return w


def test_efficiency_symmetry_rowsum(oracle_mod, mid_workload):
    """sum_i phi_i + E[f] = f(x) (the metric of the paper's stability figure);
    Phi is symmetric and its rows sum to phi."""
    ens, X = mid_workload.ensemble, mid_workload.X
    phi, Phi = oracle_mod.shap_interactions(ens, X[:4], n=32)
    fx = oracle_mod.predict(ens, X[:4])
    ev = oracle_mod.expected_value(ens)
    np.testing.assert_allclose(phi.sum(1) + ev, fx, atol=1e-12)
    np.testing.assert_allclose(Phi, np.transpose(Phi, (0, 2, 1)), atol=1e-15)
    np.testing.assert_allclose(Phi.sum(2), phi, atol=1e-12)
    phi_t = oracle_mod.treeshap(ens, X[:4])
    np.testing.assert_allclose(phi_t, phi, atol=1e-11)


def test_null_player_exact_zero(oracle_mod):
    w = synth.make_workload("c1_small", T=3, M=20, F=40)
    ens = w.ensemble
    used = np.zeros(ens.n_features, bool)
    used[ens.feature[ens.left >= 0]] = True
    assert (~used).any()
    phi, Phi = oracle_mod.shap_interactions(ens, w.X[:6])
    assert np.all(phi[:, ~used] == 0.0)
    assert np.all(Phi[:, ~used, :] == 0.0) and np.all(Phi[:, :, ~used] == 0.0)


def test_linearity_and_additivity(oracle_mod):
    w = synth.make_workload("c4_adjoint", T=6, M=8, n_train=5000)
    ens, X = w.ensemble, w.X
    phi = oracle_mod.shap_values(ens, X)
    rng = np.random.default_rng(3)
    v2 = rng.normal(size=ens.n_leaves())
    e2 = ens.with_leaf_values(v2)
    e3 = ens.with_leaf_values(2.0 * ens.leaf_values() - 0.5 * v2)
    np.testing.assert_allclose(oracle_mod.shap_values(e3, X),
                               2.0 * phi - 0.5 * oracle_mod.shap_values(e2, X), atol=1e-13)
    parts = sum(oracle_mod.shap_values(ens.subset_trees([t]), X) for t in range(ens.n_trees))
    np.testing.assert_allclose(parts, phi, atol=1e-14)


def test_duplicated_subtrees_make_a_dummy(oracle_mod):
    """If both children of a split on feature j carry identical subtrees and
    covers are additive, the game does not depend on j, so phi_j = 0."""
    sub = lambda c: ("split", 1, 0.5, c, ("leaf", 2.0, 0.25 * c), ("leaf", -1.0, 0.75 * c))
    ens = synth.from_nested([("split", 0, 0.0, 100.0, sub(30.0), sub(70.0))], n_features=2)
    X = np.array([[-1, 0], [1, 1], [0.2, 0.7]], np.float32)
    phi, Phi = oracle_mod.shap_interactions(ens, X)
    np.testing.assert_allclose(phi[:, 0], 0.0, atol=1e-15)
    np.testing.assert_allclose(Phi[:, 0, :], 0.0, atol=1e-15)


@pytest.mark.parametrize("layout", ["depth_first", "breadth_first", "grown"])
def test_leaf_gradient_is_transposed_jacobian(oracle_mod, layout):
    """phi is linear in the leaf values, so its Jacobian column for a leaf is
    phi of the model with that leaf set to 1 and all others 0; compare
    J^T G against that, column by column, from subset enumeration.  Leaves are
    indexed in tree-major node-id order; the three layouts number nodes
    depth-first, breadth-first with leaves at several depths, and depth-first
    bigger-child-first, so node-id order and visit order differ."""
    rng = np.random.default_rng(11)
    if layout == "depth_first":
        ens = synth.random_small_ensemble(rng, 2, 4, 3)
    elif layout == "breadth_first":
        ens = synth.make_workload("c2_values", T=2, M=1, n_train=300, F=5, depth=4).ensemble
        assert ens.n_leaves() < 2 * 16  # some leaves above the last level
    else:
        ens = synth.make_workload("c5_deep", T=2, M=1, n_train=400, F=5, depth=4,
                                  leaf_cap=9).ensemble
    F = ens.n_features
    X = (np.round(rng.standard_normal((3, F)) * 2) / 2).astype(np.float32)
    G = rng.normal(size=(3, F))
    L = ens.n_leaves()
    want = np.zeros(L)
    for leaf in range(L):
        e = np.zeros(L)
        e[leaf] = 1.0
        want[leaf] = np.sum(G * brute.shap_values(ens.with_leaf_values(e), X))
    for n in (8, 32):
        np.testing.assert_allclose(oracle_mod.leaf_grad(ens, X, G, n=n), want, atol=1e-13)


def test_third_order_closed_form(oracle_mod):
    """A chain of three features, cover ratio 1/2 at every split, and a row
    that goes left everywhere.  Only the two leaves below the third split
    carry all three features, so (Theorem 1 with |S| = 3; the integrand of an
    empty product is 1, exact for every rule)
      SII_012 = 1.0 (1/2)^3 + 0.3 (1/2)(1/2)(0 - 1/2) = 0.0875,
    the same for every ordering, and 0 for any triple with feature 3."""
    node = ("split", 2, 0.0, 0.25, ("leaf", 1.0, 0.125), ("leaf", 0.3, 0.125))
    node = ("split", 1, 0.0, 0.5, node, ("leaf", -0.7, 0.25))
    node = ("split", 0, 0.0, 1.0, node, ("leaf", 0.4, 0.5))
    ens = synth.from_nested([node], n_features=4)
    X = np.full((1, 4), -1.0, np.float32)
    want = np.zeros((1, 4, 4, 4))
    for a, b, c in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        want[0, a, b, c] = 0.0875
    for n in (1, 2, 8):
        np.testing.assert_allclose(oracle_mod.shap_sii3(ens, X, n=n), want, rtol=0, atol=1e-15)
    np.testing.assert_allclose(brute.shap_sii3(ens, X), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_third_order_equals_enumeration(oracle_mod, seed):
    """Third-order indices by 8-node path quadrature (exact for paths of up to
    18 features, Theorem 2) against subset enumeration of the path-dependent
    game (Theorem 3's definition), with missing values, on small irregular
    ensembles; zero covers in one of the seeds."""
    rng = np.random.default_rng(70 + seed)
    ens = synth.random_small_ensemble(rng, 3, 6, 5, zero_cover=(seed == 2))
    X = rng.standard_normal((4, 6)).astype(np.float32)
    X[1, ::2] = np.nan
    got = oracle_mod.shap_sii3(ens, X, n=8)
    want = brute.shap_sii3(ens, X)
    assert np.abs(want).max() > 1e-3
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # symmetric in its three indices, zero wherever two coincide
    for perm in ((0, 2, 1, 3), (0, 3, 2, 1), (0, 2, 3, 1)):
        np.testing.assert_array_equal(got, np.transpose(got, perm))
    i = np.arange(6)
    assert not got[:, i, i, :].any() and not got[:, :, i, i].any()
