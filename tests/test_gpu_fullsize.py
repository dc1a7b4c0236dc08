"""Full-size workloads in the benchmark's launch configuration (autotuned
launch shapes, HIP graph replay, output buffers reused across replays),
checked against the FP64 oracle on seeded sampled rows."""
import functools
import threading

import numpy as np
import pytest

import synth
from tests.parity import TOL_FP32, TOL_FP64, check, row_normwise

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


def _spread_rows(M, n, seed):
    """n seeded rows spread over all sample blocks: the first and last rows of
    the first and last 64-sample blocks, then stratified random ones."""
    fixed = [0, 63, M - 64, M - 1]
    rng = np.random.default_rng(seed)
    edges = np.linspace(0, M, n - len(fixed) + 1).astype(np.int64)
    strat = [int(rng.integers(a, b)) for a, b in zip(edges[:-1], edges[1:])]
    return np.unique(np.array(fixed + strat, np.int64))


class _Background:
    """Runs an oracle call on the host cores while the GPU works (the C
    oracle releases the interpreter lock)."""

    def __init__(self, fn, *args, **kw):
        self.out = None
        self.exc = None

        def run():
            try:
                self.out = fn(*args, **kw)
            except BaseException as exc:  # re-raised in result()
                self.exc = exc
        self.t = threading.Thread(target=run, daemon=True)
        self.t.start()

    def result(self):
        self.t.join()
        if self.exc is not None:
            raise self.exc
        return self.out


@pytest.mark.timeout(900)
def test_interactions_full_50k(q, oracle_mod):
    """The interactions workload at its stated size: 500 grown trees (depths
    3..20, leaf cap 4096), 200 features, all 50,000 samples, Phi[50k,200,200]
    in FP32 (8.0 GB) and FP64 (16 GB), in the benchmark's launch
    configuration (autotuned, HIP graph replay, output buffers reused).
    Checked against the 8-node FP64 oracle on 16 rows spread over the sample
    blocks; phi of the interactions call against qts_shap_values (the other
    kernel) on every row; and efficiency, sum_i phi_i + E[f] = f(x), on every
    row against the oracle's prediction and expected value."""
    print("c3_interactions all 50k samples", flush=True)
    wl = _wl("c3_interactions")
    ens = wl.ensemble
    M, F = wl.X.shape[0], ens.n_features
    assert M == 50000 and F == 200
    rows = _spread_rows(M, 16, 41)
    assert len(rows) == 16
    ref = _Background(oracle_mod.shap_interactions, ens, wl.X[rows], n=8)
    pred = oracle_mod.predict(ens, wl.X)
    E = oracle_mod.expected_value(ens)
    e = q.Ensemble(ens)
    assert abs(e.expected_value - E) <= 1e-12 * max(1.0, abs(E))
    X = torch.from_numpy(wl.X).cuda()
    got = {}
    for precision, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        print("c3 full", precision, flush=True)
        e.autotune(1024, precision)
        e.set_graph_replay(True)
        Phi = torch.empty((M, F, F), dtype=dt, device="cuda")
        phi = torch.empty((M, F), dtype=dt, device="cuda")
        for _ in range(2):  # capture, then replay into the same buffers
            Phi.fill_(float("nan"))
            e.shap_interactions(X, precision, with_phi=True, out=Phi, out_phi=phi)
            torch.cuda.synchronize()
        sel = torch.from_numpy(rows).cuda()
        Phi_rows = Phi[sel].double().cpu().numpy()
        assert np.isfinite(Phi_rows).all()
        # spot-check every sample block for unwritten entries (8 GB is not copied)
        assert bool(torch.isfinite(Phi[::97]).all())
        phi_i = phi.double().cpu().numpy()
        e.set_graph_replay(False)
        del Phi
        torch.cuda.empty_cache()
        phi_v = e.shap_values(X, precision).double().cpu().numpy()
        tol = TOL_FP32 if precision == "fp32" else TOL_FP64
        err_k = row_normwise(phi_i, phi_v)
        assert err_k <= tol, ("phi: interactions vs values kernel", precision, err_k)
        # efficiency against the oracle's f(x) and E[f]; the 8-node rule is exact
        # only for d <= 16 first order, which bounds the residual far below tol
        resid = np.abs(phi_i.sum(1) + E - pred)
        scale = np.abs(phi_i).sum(1) + abs(E) + np.abs(pred)
        eff = float((resid / scale).max())
        print("c3 full %s: phi kernels %.2e, efficiency %.2e" % (precision, err_k, eff),
              flush=True)
        assert eff <= tol, ("efficiency", precision, eff)
        got[precision] = (Phi_rows, phi_i[rows])
    phi_o, Phi_o = ref.result()
    for precision, (Phi_rows, phi_rows) in got.items():
        err = check(Phi_rows, Phi_o, precision, "c3 full Phi")
        check(phi_rows, phi_o, precision, "c3 full phi")
        print("c3 full %s: Phi row-normwise %.2e on %d rows" % (precision, err, len(rows)),
              flush=True)
    e.close()


def test_deep_trees_full(q, oracle_mod):
    """100 grown trees of depth 32 (paths up to ~31 unique features, every
    bucket and the long-path interactions kernel), all 10k samples; phi on 12
    rows and Phi on 8 rows spread over the samples."""
    print("c5_deep full", flush=True)
    wl = _wl("c5_deep")
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    M = X.shape[0]
    rows = _rows(M, 8, 13)
    want = oracle_mod.shap_values(wl.ensemble, wl.X[rows], n=8)
    prow = _spread_rows(M, 8, 14)
    ref = _Background(oracle_mod.shap_interactions, wl.ensemble, wl.X[prow], n=8)
    got = {}
    for precision in ("fp32", "fp64"):
        e.autotune(M, precision)
        e.set_graph_replay(True)
        phi = e.shap_values(X, precision).double().cpu().numpy()
        check(phi[rows], want, precision, "c5 phi")
        Phi = e.shap_interactions(X, precision)
        got[precision] = Phi[torch.from_numpy(prow).cuda()].double().cpu().numpy()
        del Phi
        e.set_graph_replay(False)
    _, Phi_o = ref.result()
    for precision, G in got.items():
        check(G, Phi_o, precision, "c5 Phi")
