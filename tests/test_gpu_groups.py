"""GPU parity of multi-output ensembles (a group of trees per output, as the
per-class attributions of a multiclass model): values, pairwise interactions,
third-order indices and the leaf adjoint, per output, against the oracle's
per-group composition; launch shapes autotuned and graph replay included."""
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


CASES = [
    ("c2_values", dict(T=30, M=130, n_train=20000, groups=3)),      # full depth-8 trees
    ("c3_interactions", dict(T=9, M=70, n_train=20000, groups=3)),  # buckets/classes per group
    ("c5_deep", dict(T=4, M=40, n_train=30000, groups=3)),          # long rows
]


@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_grouped_values_interactions_adjoint(q, oracle_mod, name, over):
    print("case groups", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    ens, X = wl.ensemble, wl.X.copy()
    K, F, M = ens.n_groups, ens.n_features, X.shape[0]
    assert K == 3
    X[::9, ::4] = np.nan
    e = q.Ensemble(ens)
    assert e.n_groups == 3
    np.testing.assert_allclose(e.expected_value, oracle_mod.expected_values_grouped(ens),
                               rtol=0, atol=1e-12)
    Xd = torch.from_numpy(X).cuda()
    want = oracle_mod.shap_values_grouped(ens, X)
    pw, Pw = oracle_mod.shap_interactions_grouped(ens, X[:12])
    rng = np.random.default_rng(9)
    G = rng.standard_normal((M, K, F))
    for precision in ("fp32", "fp64"):
        for merge in (True, False):
            e.set_sibling_merge(merge)
            phi = e.shap_values(Xd, precision)
            assert tuple(phi.shape) == (M, K, F)
            check(phi.double().cpu().numpy().reshape(M * K, F), want.reshape(M * K, F),
                  precision, "%s grouped phi merge=%s" % (name, merge))
        Phi, phi_i = e.shap_interactions(Xd[:12], precision, with_phi=True)
        assert tuple(Phi.shape) == (12, K, F, F)
        check(Phi.double().cpu().numpy().reshape(12 * K, -1), Pw.reshape(12 * K, -1), precision,
              name + " grouped Phi")
        check(phi_i.double().cpu().numpy().reshape(12 * K, F), pw.reshape(12 * K, F), precision,
              name + " grouped phi (interactions)")
        Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
        gw = oracle_mod.leaf_grad_grouped(ens, X, Gp)
        gl = e.shap_backward(Xd, torch.from_numpy(Gp).cuda(), precision).cpu().numpy()
        err = float(np.abs(gl - gw).max() / np.abs(gw).max())
        assert err <= (1e-5 if precision == "fp32" else 1e-10), (precision, err)


def test_grouped_third_order_and_replay(q, oracle_mod):
    wl = synth.make_workload("c4_adjoint", T=9, M=11, n_train=20000, F=12, groups=3)
    ens, X = wl.ensemble, wl.X
    e = q.Ensemble(ens)
    Xd = torch.from_numpy(X).cuda()
    want3 = oracle_mod.shap_sii3_grouped(ens, X)
    for precision in ("fp32", "fp64"):
        t3 = e.shap_interactions3(Xd, precision)
        assert tuple(t3.shape) == (11, 3, 12 * 11 * 10 // 6)
        dense = e.triples_dense(t3, 12).double().cpu().numpy()
        check(dense.reshape(33, -1), want3.reshape(33, -1), precision, "grouped third order")
    # autotuned shapes and graph replay into reused buffers
    want = oracle_mod.shap_values_grouped(ens, X)
    e.autotune(64, "fp32")
    e.set_graph_replay(True)
    out = torch.empty((11, 3, 12), device="cuda")
    for _ in range(3):
        out.fill_(float("nan"))
        e.shap_values(Xd, "fp32", out=out)
        torch.cuda.synchronize()
        check(out.double().cpu().numpy().reshape(33, 12), want.reshape(33, 12), "fp32",
              "grouped replay")
    e.set_graph_replay(False)


def test_grouped_wide_feature_space(q, oracle_mod):
    """300 features (the first-order kernels take segments, X and grad_phi
    feature-major, an accumulator [K][F][M] transposed into phi [M][K][F]) with
    two outputs: values and the adjoint, both precisions, eager, graph replay
    and the deterministic mode, against the oracle's per-group composition."""
    wl = synth.make_workload("c2_values", F=300, T=24, M=150, n_train=20000, groups=2)
    ens, X = wl.ensemble, wl.X.copy()
    K, F, M = ens.n_groups, ens.n_features, X.shape[0]
    X[::7, ::5] = np.nan
    e = q.Ensemble(ens)
    assert e.info["n_value_segments"] > 0
    Xd = torch.from_numpy(X).cuda()
    want = oracle_mod.shap_values_grouped(ens, X)
    G = np.random.default_rng(31).standard_normal((M, K, F))
    for mode in ("eager", "replay", "deterministic"):
        e.set_graph_replay(mode == "replay")
        e.set_deterministic(mode == "deterministic")
        for precision in ("fp32", "fp64"):
            for _ in range(2 if mode == "replay" else 1):
                phi = e.shap_values(Xd, precision)
                check(phi.double().cpu().numpy().reshape(M * K, F), want.reshape(M * K, F),
                      precision, "wide grouped phi %s" % mode)
                Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
                gw = oracle_mod.leaf_grad_grouped(ens, X, Gp)
                gl = e.shap_backward(Xd, torch.from_numpy(Gp).cuda(), precision).cpu().numpy()
                err = float(np.abs(gl - gw).max() / np.abs(gw).max())
                assert err <= (1e-5 if precision == "fp32" else 1e-10), (mode, precision, err)
    e.set_graph_replay(False)
    e.set_deterministic(False)

