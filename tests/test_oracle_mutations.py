"""Planted-mistake check for the oracle pins (CPU only).

Each case compiles a copy of the oracle source with one plausible mistake
(a dropped term, a wrong sign, a swapped operand, a wrong index, a wrong
routing rule) and requires the pins — closed forms, enumeration of the
definitions, quadrature exactness — to reject it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import brute
from oracle import oracle as O

SRC = os.path.join(os.path.dirname(O.__file__), "qts_oracle.c")

MUTATIONS = {
    "sign_of_o_minus_b": ("double coef = (o[i] - b[i]) * integral;",
                          "double coef = (b[i] - o[i]) * integral;"),
    "dropped_follow_term": ("return b * s + o * t;", "return b * s;"),
    # (b t + o s is an equivalent mutant: the rule is symmetric under t -> 1-t)
    "follow_term_uses_s": ("return b * s + o * t;", "return b * s + o * s;"),
    "leave_one_out_index": ("if (j != i) prod *= factor", "if (j != d - 1 - i) prod *= factor"),
    "weight_scale": ("omega[i] = 1.0 / ((1.0 - x * x) * dp * dp);",
                     "omega[i] = 2.0 / ((1.0 - x * x) * dp * dp);"),
    "collapse_last_edge_wins": ("o[k] *= e[i].sat ? 1.0 : 0.0;", "o[k] = e[i].sat ? 1.0 : 0.0;"),
    "collapse_b_not_product": ("b[k] *= e[i].w;", "b[k] = e[i].w;"),
    "pair_uses_i_twice": ("val * (o[i] - b[i]) * (o[k] - b[k]) * integral",
                          "val * (o[i] - b[i]) * (o[i] - b[i]) * integral"),
    "pair_drops_k_not_i": ("if (j != i && j != k) prod", "if (j != i) prod"),
    "ties_go_left": ("return xv < m->threshold[g];", "return xv <= m->threshold[g];"),
    "nan_wrong_direction": ("return m->default_left[g] != 0;", "return m->default_left[g] == 0;"),
    "edge_weight_of_parent": ("return m->cover[child] / cp;", "return m->cover[child] / (cp + 1.0);"),
    "leaf_ordinal_in_visit_order": ("leaf_ordinal(m, base, node));", "(*leaf_ord)++);"),
    "triple_drops_k": ("if (l != i && l != j && l != k) prod *=", "if (l != i && l != j) prod *="),
    "triple_uses_j_twice": ("(o[i] - b[i]) * (o[j] - b[j]) * (o[k] - b[k]) * integral",
                            "(o[i] - b[i]) * (o[j] - b[j]) * (o[j] - b[j]) * integral"),
    "triple_ordering_missing": ("        c->sii3[(z * F + y) * F + x] += v;\n", ""),
}


def _pins_pass() -> bool:
    """The oracle pins of test_oracle.py in compact form; True when all hold."""
    try:
        # quadrature rule exactness
        t, s, w = O.gauss_legendre(8)
        for k in range(16):
            if abs(np.sum(w * t ** k) - 1.0 / (k + 1)) > 1e-13:
                return False
        # stump closed form
        st = synth.stump()
        if not np.allclose(O.shap_values(st, np.array([[-1.0], [0.0]], np.float32)),
                           [[2.1], [-0.9]], atol=1e-13):
            return False
        if abs(O.expected_value(st) + 1.1) > 1e-13:
            return False
        # enumeration of the definitions, with ties and missing values
        for seed in range(3):
            rng = np.random.default_rng(100 + seed)
            ens = synth.random_small_ensemble(rng, 3, 6, 5)
            X = (np.round(rng.standard_normal((5, 6)) * 2) / 2).astype(np.float32)
            X[0, rng.integers(6)] = np.nan
            X[1, :] = np.nan
            phi_q, sii_q = O.shap_sii(ens, X, n=8)
            if not np.allclose(phi_q, brute.shap_values(ens, X), atol=1e-12):
                return False
            if not np.allclose(sii_q, brute.shap_sii(ens, X), atol=1e-12):
                return False
            if not np.allclose(O.shap_sii3(ens, X, n=8), brute.shap_sii3(ens, X), atol=1e-12):
                return False
            G = rng.normal(size=(5, 6))
            J = np.zeros(ens.n_leaves())
            for leaf in range(ens.n_leaves()):
                e = np.zeros(ens.n_leaves())
                e[leaf] = 1.0
                J[leaf] = np.sum(G * brute.shap_values(ens.with_leaf_values(e), X))
            if not np.allclose(O.leaf_grad(ens, X, G), J, atol=1e-12):
                return False
        # leaf order on a breadth-first tree with leaves at several depths
        ens = synth.make_workload("c2_values", T=2, M=1, n_train=300, F=5, depth=4).ensemble
        X = np.random.default_rng(8).standard_normal((3, 5)).astype(np.float32)
        G = np.random.default_rng(9).normal(size=(3, 5))
        J = np.zeros(ens.n_leaves())
        for leaf in range(ens.n_leaves()):
            e = np.zeros(ens.n_leaves())
            e[leaf] = 1.0
            J[leaf] = np.sum(G * brute.shap_values(ens.with_leaf_values(e), X))
        if not np.allclose(O.leaf_grad(ens, X, G), J, atol=1e-12):
            return False
        return True
    except (RuntimeError, ValueError, FloatingPointError):
        return False


def test_unmodified_oracle_passes_pins(oracle_mod):
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, monkeypatch, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor missing: " + name
    bad = tmp_path / "mutant.c"
    bad.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-shared", "-fPIC",
                           "-pthread", "-o", str(so), str(bad), "-lm"])
    L = ctypes.CDLL(str(so))
    for fn in ("orc_gauss_legendre", "orc_shap_values", "orc_shap_interactions",
               "orc_leaf_grad", "orc_expected_value", "orc_predict", "orc_treeshap",
               "orc_shap_sii3"):
        getattr(L, fn).restype = ctypes.c_int
    monkeypatch.setattr(O, "_lib", L)
    with np.errstate(all="ignore"):
        assert not _pins_pass(), "pins did not catch: " + name
