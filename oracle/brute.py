"""Brute-force Shapley values and Shapley interaction indices by subset
enumeration, straight from their definitions.

TEST INFRASTRUCTURE ONLY (see oracle.py).  Written in numpy, independently of
the C oracle: it evaluates the path-dependent game v_x(S) leaf by leaf and
enumerates coalitions.  Usable only on tiny models (a few features per tree).

Game (Eq. 1-3): for a leaf v with path edges e and a coalition S,
  f_v(S) = val(v) * prod_e ( f(e) in S ? 1[x satisfies e] : w_e ),
which equals R_empty * prod_{i in S} q_i with q_i as in Eq. 2.  The tree's game
is the sum over its leaves; the ensemble's the sum over trees.

Shapley interaction index (Theorem 3, Appendix D), for |S| = s:
  SII(S) = sum_{T subset of [F] minus S} |T|! (F-s-|T|)! / (F-s+1)!  Delta_S v(T),
  Delta_S v(T) = sum_{L subset of S} (-1)^{s-|L|} v(T union L)         (Def. 1)
with s = 1 the Shapley value.  Features absent from a tree are null players
of that tree's game (Lemma 2, case 1), so each tree is enumerated over its own
features only and the results are added over trees.
"""
from __future__ import annotations

import itertools
from math import factorial

import numpy as np


def _paths(ens, t):
    """Yield (leaf value, [(feature, w_e, is_left_edge, threshold, default_left)])."""
    a = int(ens.tree_offsets[t])
    stack = [(0, [])]
    while stack:
        node, edges = stack.pop()
        g = a + node
        if ens.left[g] < 0:
            yield float(ens.value[g]), edges
            continue
        cp = float(ens.cover[g])
        for child, is_left in ((int(ens.left[g]), True), (int(ens.right[g]), False)):
            w = 0.0 if cp == 0.0 else float(ens.cover[a + child]) / cp
            stack.append((child, edges + [(int(ens.feature[g]), w, is_left,
                                           np.float32(ens.threshold[g]),
                                           bool(ens.default_left[g]))]))


def _satisfies(xv, is_left, thr, default_left):
    if np.isnan(xv):
        return is_left == default_left
    goes_left = np.float32(xv) < thr
    return goes_left if is_left else not goes_left


def tree_game(ens, t, x):
    """Return (features of tree t, v) with v(frozenset S) the tree's game."""
    paths = list(_paths(ens, t))
    feats = sorted({e[0] for _, edges in paths for e in edges})
    sat = [[_satisfies(x[e[0]], e[2], e[3], e[4]) for e in edges] for _, edges in paths]

    def v(S):
        total = 0.0
        for (val, edges), ss in zip(paths, sat):
            prod = val
            for e, s in zip(edges, ss):
                prod *= (1.0 if s else 0.0) if e[0] in S else e[1]
            total += prod
        return total

    return feats, v


def _sii_of_game(feats, v, order):
    """SII for all ordered `order`-subsets of feats, over the game's own players."""
    n = len(feats)
    cache = {}

    def val(S):
        key = frozenset(S)
        if key not in cache:
            cache[key] = v(key)
        return cache[key]

    out = {}
    for S in itertools.combinations(feats, order):
        rest = [f for f in feats if f not in S]
        s = len(S)
        total = 0.0
        for r in range(len(rest) + 1):
            wgt = factorial(r) * factorial(n - s - r) / factorial(n - s + 1)
            for T in itertools.combinations(rest, r):
                delta = 0.0
                for ell in range(s + 1):
                    for L in itertools.combinations(S, ell):
                        delta += (-1) ** (s - ell) * val(T + L)
                total += wgt * delta
        out[S] = total
    return out


def shap_values(ens, X):
    """phi[M,F] by enumeration (Shapley values of the path-dependent game)."""
    X = np.asarray(X, np.float32)
    phi = np.zeros((X.shape[0], ens.n_features))
    for r in range(X.shape[0]):
        for t in range(ens.n_trees):
            feats, v = tree_game(ens, t, X[r])
            for (i,), val in _sii_of_game(feats, v, 1).items():
                phi[r, i] += val
    return phi


def shap_sii(ens, X):
    """sii[M,F,F] for ordered pairs i != k by enumeration (diagonal 0)."""
    X = np.asarray(X, np.float32)
    F = ens.n_features
    sii = np.zeros((X.shape[0], F, F))
    for r in range(X.shape[0]):
        for t in range(ens.n_trees):
            feats, v = tree_game(ens, t, X[r])
            for (i, k), val in _sii_of_game(feats, v, 2).items():
                sii[r, i, k] += val
                sii[r, k, i] += val
    return sii


def shap_sii3(ens, X):
    """sii3[M,F,F,F] for ordered triples of distinct features by enumeration."""
    X = np.asarray(X, np.float32)
    F = ens.n_features
    sii3 = np.zeros((X.shape[0], F, F, F))
    for r in range(X.shape[0]):
        for t in range(ens.n_trees):
            feats, v = tree_game(ens, t, X[r])
            for S, val in _sii_of_game(feats, v, 3).items():
                for a, b, c in itertools.permutations(S):
                    sii3[r, a, b, c] += val
    return sii3


def game_value(ens, x, S):
    """Ensemble game v_x(S) (sum over trees)."""
    return sum(tree_game(ens, t, x)[1](frozenset(S)) for t in range(ens.n_trees))
