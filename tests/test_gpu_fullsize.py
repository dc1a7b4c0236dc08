"""Full-size workloads in the benchmark's launch configuration (autotuned
launch shapes, HIP graph replay, output buffers reused across replays),
checked against the FP64 oracle on seeded sampled rows."""
import functools

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


@functools.lru_cache(maxsize=1)
def _wl(name):
    return synth.make_workload(name)


def _rows(M, n, seed):
    r = np.random.default_rng(seed).choice(M, n, replace=False)
    return np.unique(np.concatenate([r, [0, 63, 64, M - 1]]))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_values_headline_bench_config(q, oracle_mod, precision):
    """1000 random trees of depth 8, 100 features, 100k samples."""
    print("c2_values full, bench configuration", precision, flush=True)
    wl = _wl("c2_values")
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    M = X.shape[0]
    e.autotune(M, precision)
    e.set_graph_replay(True)
    out = torch.empty((M, e.n_features), dtype=torch.float32 if precision == "fp32"
                      else torch.float64, device="cuda")
    rows = _rows(M, 16, 11)
    want = oracle_mod.shap_values(wl.ensemble, wl.X[rows], n=8)
    for _ in range(2):  # capture, then replay
        out.zero_()
        e.shap_values(X, precision, out=out)
        torch.cuda.synchronize()
        check(out.double().cpu().numpy()[rows], want, precision, "c2 full")


def test_interactions_bench_config(q, oracle_mod):
    """500 grown trees (depths 3..20), 200 features: the first 1024 samples,
    as timed by the benchmark, in FP32 and FP64."""
    print("c3_interactions full ensemble, 1024 samples", flush=True)
    wl = _wl("c3_interactions")
    e = q.Ensemble(wl.ensemble)
    M = 1024
    X = torch.from_numpy(wl.X[:M]).cuda()
    rows = np.array([0, 517, M - 1])
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X[rows], n=8)
    for precision, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        e.autotune(M, precision)
        e.set_graph_replay(True)
        Phi = torch.empty((M, e.n_features, e.n_features), dtype=dt, device="cuda")
        phi = torch.empty((M, e.n_features), dtype=dt, device="cuda")
        for _ in range(2):
            e.shap_interactions(X, precision, with_phi=True, out=Phi, out_phi=phi)
            torch.cuda.synchronize()
            check(Phi[rows].double().cpu().numpy(), Phi_o, precision, "c3 Phi")
            check(phi[rows].double().cpu().numpy(), phi_o, precision, "c3 phi")
        e.set_graph_replay(False)
        del Phi, phi


def test_deep_trees_full(q, oracle_mod):
    """100 grown trees of depth 32 (paths up to ~31 unique features, every
    bucket and the long-path interactions kernel), all 10k samples."""
    print("c5_deep full", flush=True)
    wl = _wl("c5_deep")
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    M = X.shape[0]
    rows = _rows(M, 8, 13)
    want = oracle_mod.shap_values(wl.ensemble, wl.X[rows], n=8)
    prow = rows[:2]
    _, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X[prow], n=8)
    for precision in ("fp32", "fp64"):
        e.autotune(M, precision)
        e.set_graph_replay(True)
        phi = e.shap_values(X, precision).double().cpu().numpy()
        check(phi[rows], want, precision, "c5 phi")
        Phi = e.shap_interactions(X[:2048], precision)
        check(Phi[torch.from_numpy(prow).cuda()].double().cpu().numpy(), Phi_o, precision,
              "c5 Phi")
        e.set_graph_replay(False)
