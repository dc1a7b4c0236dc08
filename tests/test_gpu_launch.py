"""Batching and launch: the launch-shape autotuner and HIP graph replay.

Every tuned shape must keep parity with the FP64 oracle, and every graph
replay must equal the eager call on the same inputs, replay after replay, with
other eager GPU work and host synchronisations in between (a graph reads its
input buffers at replay time, so new contents of the same X must show)."""
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


VALUES_WAVES = {4, 6, 8}
VALUES_ITEMS = {4096, 8192, 16384, 32768, 65536}
PAIR_CHUNKS = {8192, 32768, 131072}
PAIR_FILL = {1024, 4096}


def test_default_shapes(q):
    wl = synth.make_workload("c1_small", M=8)
    e = q.Ensemble(wl.ensemble)
    assert e.launch_shape("values", "fp32", 0) == (8, 16384)
    assert e.launch_shape("interactions", "fp32", 0) == (65536, 2048)
    assert e.launch_shape("adjoint", "fp32", 0) == (8, 16384)
    with pytest.raises(q.QtsError):
        e.launch_shape("values", "fp32", 4)


@pytest.mark.parametrize("name,over", [
    ("c2_values", dict(T=40, M=3000, n_train=20000)),
    ("c5_deep", dict(T=3, M=200, n_train=30000)),      # buckets 8..64 and long classes
])
def test_autotune_keeps_parity(q, oracle_mod, name, over):
    print("case", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    rows = slice(0, 24)
    phi_o, Phi_o = oracle_mod.shap_interactions(wl.ensemble, wl.X[rows], n=8)
    want = oracle_mod.shap_values(wl.ensemble, wl.X, n=8)
    for precision in ("fp32", "fp64"):
        e.autotune(wl.X.shape[0], precision)
        for i in range(4):
            for kind in ("values", "adjoint"):
                w, items = e.launch_shape(kind, precision, i)
                assert w in VALUES_WAVES and items in VALUES_ITEMS, (kind, w, items)
        for i in range(e.info["n_pair_classes"]):
            mc, fill = e.launch_shape("interactions", precision, i)
            assert mc in PAIR_CHUNKS and fill in PAIR_FILL, (mc, fill)
        phi = e.shap_values(X, precision).double().cpu().numpy()
        check(phi, want, precision, name + " tuned phi")
        Phi = e.shap_interactions(X[rows], precision).double().cpu().numpy()
        check(Phi, Phi_o, precision, name + " tuned Phi")


def _eager_values(q, ens, X, precision):
    e = q.Ensemble(ens)
    out = e.shap_values(X, precision).clone()
    e.close()
    return out


@pytest.mark.parametrize("name,over", [
    ("c1_small", dict(M=300)),
    ("c5_deep", dict(T=3, M=150, n_train=30000)),     # four buckets: parallel branches
])
def test_graph_replay_values(q, oracle_mod, name, over):
    print("case", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    e.set_graph_replay(True)
    X = torch.from_numpy(wl.X).cuda()
    rng = np.random.default_rng(5)
    X2h = rng.standard_normal(wl.X.shape).astype(np.float32)
    for precision in ("fp32", "fp64"):
        out = torch.empty((X.shape[0], e.n_features), dtype=torch.float32 if precision == "fp32"
                          else torch.float64, device="cuda")
        ref1 = _eager_values(q, wl.ensemble, X, precision)
        ref2 = _eager_values(q, wl.ensemble, torch.from_numpy(X2h).cuda(), precision)
        Xbuf = X.clone()
        n0 = e.refresh_info()["n_graphs"]
        tol = 1e-6 if precision == "fp32" else 1e-13
        for rep in range(4):
            # eager GPU work and a host synchronisation between replays
            junk = torch.randn(1 << 16, device="cuda").cumsum(0)
            torch.cuda.synchronize()
            if rep == 2:                       # same buffer, new contents
                Xbuf.copy_(torch.from_numpy(X2h).cuda())
            e.shap_values(Xbuf, precision, out=out)
            torch.cuda.synchronize()
            ref = ref2 if rep >= 2 else ref1
            assert row_normwise(out.double().cpu().numpy(), ref.double().cpu().numpy()) <= tol
            del junk
        assert e.refresh_info()["n_graphs"] == n0 + 1   # captured once, replayed after
        check(out.double().cpu().numpy(), oracle_mod.shap_values(wl.ensemble, X2h, n=8),
              precision, name + " replay vs oracle")
    e.set_graph_replay(False)
    assert e.refresh_info()["n_graphs"] == 0


def test_graph_replay_interactions_and_backward(q, oracle_mod):
    wl = synth.make_workload("c3_interactions", T=4, M=20, n_train=20000)
    ens = wl.ensemble
    e = q.Ensemble(ens)
    X = torch.from_numpy(wl.X).cuda()
    phi_o, Phi_o = oracle_mod.shap_interactions(ens, wl.X, n=8)
    G = np.random.default_rng(8).normal(size=(wl.X.shape[0], ens.n_features))
    e.set_graph_replay(True)
    for precision in ("fp32", "fp64"):
        dt = torch.float32 if precision == "fp32" else torch.float64
        Phi = torch.empty((X.shape[0], e.n_features, e.n_features), dtype=dt, device="cuda")
        phi = torch.empty((X.shape[0], e.n_features), dtype=dt, device="cuda")
        Gd = torch.from_numpy(G).cuda().to(dt)
        gl = torch.empty(e.n_leaves, dtype=torch.float64, device="cuda")
        Gw = Gd.double().cpu().numpy()
        want_g = oracle_mod.leaf_grad(ens, wl.X, Gw)
        for rep in range(3):
            torch.randn(4096, device="cuda").sum()
            torch.cuda.synchronize()
            e.shap_interactions(X, precision, with_phi=True, out=Phi, out_phi=phi)
            e.shap_backward(X, Gd, precision, out=gl)
            torch.cuda.synchronize()
            check(Phi.double().cpu().numpy(), Phi_o, precision, "replay Phi %d" % rep)
            check(phi.double().cpu().numpy(), phi_o, precision, "replay phi %d" % rep)
            g = gl.cpu().numpy()
            err = np.abs(g - want_g).max() / np.abs(want_g).max()
            assert err <= (1e-5 if precision == "fp32" else 1e-10), err
    assert e.refresh_info()["n_graphs"] == 4


def test_graph_replay_third_order(q, oracle_mod):
    """qts_shap_interactions3 under graph replay, in both traversals and
    precisions: each key is captured once and replayed with other eager GPU
    work and host synchronisations in between; every replay matches the
    oracle and the eager call (up to the order of FP64 atomic additions); a
    leaf-value override is a key of its own."""
    wl = synth.make_workload("c5_deep", T=3, M=9, n_train=30000)
    ens = wl.ensemble
    e = q.Ensemble(ens)
    X = torch.from_numpy(wl.X).cuda()
    F = ens.n_features
    T3 = F * (F - 1) * (F - 2) // 6
    dense = oracle_mod.shap_sii3(ens, wl.X, n=8)
    idx = np.array([(i, j, k) for k in range(F) for j in range(k) for i in range(j)])
    want = dense[:, idx[:, 0], idx[:, 1], idx[:, 2]]
    lv = np.random.default_rng(12).normal(size=ens.n_leaves())
    dense_lv = oracle_mod.shap_sii3(ens.with_leaf_values(lv), wl.X, n=8)
    want_lv = dense_lv[:, idx[:, 0], idx[:, 1], idx[:, 2]]
    lvd = torch.from_numpy(lv).cuda()
    for trav in ("paths", "dfs"):
        e.set_pair_traversal(trav)
        for precision in ("fp32", "fp64"):
            dt = torch.float32 if precision == "fp32" else torch.float64
            eager = e.shap_interactions3(X, precision).cpu().numpy()
            check(eager.astype(np.float64), want, precision, "eager %s" % trav)
            out = torch.empty((X.shape[0], T3), dtype=dt, device="cuda")
            out_lv = torch.empty_like(out)
            e.set_graph_replay(True)
            n0 = e.refresh_info()["n_graphs"]
            for rep in range(3):
                torch.randn(4096, device="cuda").sum()
                torch.cuda.synchronize()
                out.fill_(float("nan"))
                e.shap_interactions3(X, precision, out=out)
                e.shap_interactions3(X, precision, leaf_values=lvd, out=out_lv)
                torch.cuda.synchronize()
                # the same kernels as the eager call; FP64 atomics may add in
                # another order, so the two agree up to rounding
                got = out.cpu().numpy().astype(np.float64)
                scale = np.abs(eager).max()
                tol = 1e-6 if precision == "fp32" else 1e-12
                assert np.abs(got - eager).max() <= tol * scale, (trav, precision, rep)
                check(got, want, precision, "replay %s %d" % (trav, rep))
                check(out_lv.double().cpu().numpy(), want_lv, precision,
                      "replay leaf override %s %d" % (trav, rep))
            assert e.refresh_info()["n_graphs"] == n0 + 2
            e.set_graph_replay(False)


def test_graph_cache_eviction(q, oracle_mod):
    """More keys than the cache holds: the least recently used graphs are
    dropped and every call still returns the right result."""
    wl = synth.make_workload("c1_small", M=40)
    e = q.Ensemble(wl.ensemble)
    e.set_graph_replay(True)
    X = torch.from_numpy(wl.X).cuda()
    want = oracle_mod.shap_values(wl.ensemble, wl.X, n=8)
    for k in range(20):
        m = 20 + k            # a new (M) key each time
        out = e.shap_values(X[:m], "fp64")
        torch.cuda.synchronize()
        assert row_normwise(out.cpu().numpy(), want[:m]) <= 1e-10
    assert e.refresh_info()["n_graphs"] == 16


def test_shapes_kept_per_node_policy(q):
    """First-order and adjoint launch shapes are tuned and kept per node
    policy: tuning under one policy leaves the other's shapes alone."""
    wl = synth.make_workload("c2_values", T=10, M=500, n_train=20000)
    e = q.Ensemble(wl.ensemble)
    kinds = ("values", "adjoint")
    e.autotune(500, "fp32")
    tuned8 = [e.launch_shape(k, "fp32", 0) for k in kinds]
    e.set_node_policy("exact")
    assert [e.launch_shape(k, "fp32", 0) for k in kinds] == [(8, 16384)] * 2  # untuned
    e.autotune(500, "fp32")
    for k in kinds:
        w, items = e.launch_shape(k, "fp32", 0)
        assert w in VALUES_WAVES and items in VALUES_ITEMS
    e.set_node_policy("fixed8")
    assert [e.launch_shape(k, "fp32", 0) for k in kinds] == tuned8


def test_calls_on_side_streams(q, oracle_mod):
    """Calls made under a non-default torch stream (default priority) run on
    that stream, eager and under graph replay: two ensembles alternate
    between two streams, with new X contents between rounds, and every
    result matches the oracle."""
    wl = synth.make_workload("c1_small", M=300)
    X2 = wl.X[::-1].copy()
    want = [oracle_mod.shap_values(wl.ensemble, x, n=8) for x in (wl.X, X2)]
    _, want_pairs = oracle_mod.shap_interactions(wl.ensemble, wl.X[:8], n=8)
    e1, e2 = q.Ensemble(wl.ensemble), q.Ensemble(wl.ensemble)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    X = torch.from_numpy(wl.X).cuda()
    torch.cuda.synchronize()
    for replay in (False, True):
        e1.set_graph_replay(replay)
        e2.set_graph_replay(replay)
        for it in range(4):
            k = it % 2
            X.copy_(torch.from_numpy(wl.X if k == 0 else X2))
            torch.cuda.synchronize()
            with torch.cuda.stream(s1):
                a = e1.shap_values(X, "fp64")
            with torch.cuda.stream(s2):
                b = e2.shap_values(X, "fp32")
                P = e2.shap_interactions(X[:8], "fp64")
            s1.synchronize()
            s2.synchronize()
            check(a.cpu().numpy(), want[k], "fp64", "stream 1, replay %s, round %d" % (replay, it))
            check(b.double().cpu().numpy(), want[k], "fp32",
                  "stream 2, replay %s, round %d" % (replay, it))
            if k == 0:
                check(P.cpu().numpy(), want_pairs, "fp64", "stream 2 pairs, replay %s" % replay)
    e1.close()
    e2.close()


def test_autotune_cache_round_trip(q, oracle_mod, tmp_path):
    """A tuned shape is written to the cache file and served from it to the
    next ensemble of the same table without timing; a cache hit keeps
    parity."""
    path = tmp_path / "tune.txt"
    wl = synth.make_workload("c2_values", T=12, M=300, n_train=20000)
    try:
        q.set_tune_cache(str(path))
        e1 = q.Ensemble(wl.ensemble)
        e1.autotune(300, "fp32")
        h1, m1 = q.tune_cache_stats()
        assert h1 == 0 and m1 > 0
        lines = path.read_text().splitlines()
        assert len(lines) == m1 and all(" -> " in ln for ln in lines)
        assert any("kind=values" in ln for ln in lines) and any("kind=pairs" in ln
                                                                 for ln in lines)
        e2 = q.Ensemble(wl.ensemble)
        e2.autotune(300, "fp32")
        h2, m2 = q.tune_cache_stats()
        assert h2 == m1 and m2 == m1          # every lookup of the second tuning hit
        assert len(path.read_text().splitlines()) == m1
        for kind, n in (("values", 1), ("adjoint", 1), ("interactions", e1.info["n_pair_classes"])):
            for i in range(n):
                assert e1.launch_shape(kind, "fp32", i) == e2.launch_shape(kind, "fp32", i)
        X = torch.from_numpy(wl.X).cuda()
        check(e2.shap_values(X, "fp32").double().cpu().numpy(),
              oracle_mod.shap_values(wl.ensemble, wl.X, n=8), "fp32", "cached shapes")
    finally:
        q.set_tune_cache(None)


@pytest.mark.parametrize("name,over", [
    ("c2_values", dict(T=40, M=900, n_train=20000)),          # one bucket, many chunks
    ("c5_deep", dict(T=3, M=300, n_train=30000)),             # several buckets
    ("c2_values", dict(F=784, T=8, M=200, n_train=20000)),    # feature segments
])
def test_deterministic_mode_bitwise(q, oracle_mod, name, over):
    """With the deterministic setting, phi and grad_leaf are identical bit for
    bit across repeated calls (eager and replayed, with other launches in
    between), and still match the oracle."""
    print("case deterministic", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    e.autotune(wl.X.shape[0], "fp64")
    e.set_deterministic(True)
    X = torch.from_numpy(wl.X).cuda()
    G = torch.from_numpy(np.random.default_rng(8).standard_normal(
        (wl.X.shape[0], e.n_features))).cuda()
    want = oracle_mod.shap_values(wl.ensemble, wl.X, n=8)
    gwant = oracle_mod.leaf_grad(wl.ensemble, wl.X, G.cpu().numpy())
    for precision in ("fp64", "fp32"):
        Gp = G if precision == "fp64" else G.float()
        runs, gruns = [], []
        for i in range(4):
            e.set_graph_replay(i >= 2)
            runs.append(e.shap_values(X, precision).cpu())
            gruns.append(e.shap_backward(X, Gp, precision).cpu())
            torch.cuda.synchronize()
            e.shap_values(X[: 1 + i], precision)  # other work in between
        for r in runs[1:]:
            assert torch.equal(r, runs[0]), precision
        for g in gruns[1:]:
            assert torch.equal(g, gruns[0]), precision
        check(runs[0].double().numpy(), want, precision, "deterministic phi")
        gw = gwant if precision == "fp64" else oracle_mod.leaf_grad(
            wl.ensemble, wl.X, Gp.double().cpu().numpy())
        err = float(np.abs(gruns[0].numpy() - gw).max() / np.abs(gw).max())
        assert err <= (1e-5 if precision == "fp32" else 1e-10), err
        e.set_graph_replay(False)
    e.close()
