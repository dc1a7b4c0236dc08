"""GPU parity of the adjoint qts_shap_backward (grad_leaf = J^T G, phi linear in
the leaf values) against the oracle's transposed map, against central finite
differences of L = ||phi - target||^2 on the full adjoint workload, and
through the torch.autograd wrapper."""
import functools

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def q():
    import paper_2605_04497_amd as q
    return q


def normwise(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


TOL = {"fp32": 1e-5, "fp64": 1e-10}


@functools.lru_cache(maxsize=1)
def _full_c4():
    return synth.make_workload("c4_adjoint")


CASES = [
    ("c4_adjoint", dict(T=20, M=500, n_train=20000)),
    ("c2_values", dict(T=10, M=300, n_train=20000)),
    ("c5_deep", dict(T=2, M=100, n_train=30000)),   # long paths (16/32/64 buckets)
    ("c1_small", dict()),
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_oracle(q, oracle_mod, name, over, precision):
    print("case", name, over, precision, flush=True)
    wl = synth.make_workload(name, **over)
    rng = np.random.default_rng(17)
    G = rng.normal(size=wl.X.shape[:1] + (wl.ensemble.n_features,))
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    g = e.shap_backward(X, torch.from_numpy(G).cuda(), precision).cpu().numpy()
    want = oracle_mod.leaf_grad(wl.ensemble, wl.X, G.astype(np.float32).astype(np.float64)
                                if precision == "fp32" else G)
    assert normwise(g, want) <= TOL[precision], normwise(g, want)


def test_full_workload_transposed_map(q, oracle_mod):
    """All 12,800 leaf gradients of the full adjoint workload (200 full trees
    of depth 6, all 20k samples, G = dL/dphi of L = ||phi - target||^2 at
    phi = 0) against the oracle's J^T G, in both precisions, eager and under
    graph replay."""
    wl = _full_c4()
    assert wl.ensemble.n_leaves() == 12800 and wl.X.shape[0] == 20000
    G = 2.0 * (np.zeros((wl.X.shape[0], wl.ensemble.n_features)) - wl.target)
    e = q.Ensemble(wl.ensemble)
    want = oracle_mod.leaf_grad(wl.ensemble, wl.X, G)
    X = torch.from_numpy(wl.X).cuda()
    Gd = torch.from_numpy(G).cuda()
    for replay in (False, True):
        e.set_graph_replay(replay)
        for precision in ("fp32", "fp64"):
            out = torch.empty(e.n_leaves, dtype=torch.float64, device="cuda")
            for _ in range(2 if replay else 1):
                g = e.shap_backward(X, Gd, precision, out=out).cpu().numpy()
                err = normwise(g, want)
                print("c4 J^T G all leaves, all samples: %s replay=%s err %.2e" % (
                    precision, replay, err), flush=True)
                assert err <= TOL[precision]
    e.close()


def test_full_workload_central_differences(q):
    """dL/dval for L = ||phi - target||^2 on the full workload (20k samples)
    against central differences with h = 1e-6 in FP64 on 256 seeded leaves.
    phi is linear in the leaf values, so L is quadratic and the central
    difference has no truncation error, only rounding (~1e-16 |L| / h)."""
    wl = _full_c4()
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    target = torch.from_numpy(wl.target.astype(np.float64)).cuda()
    v0 = torch.from_numpy(wl.ensemble.leaf_values()).cuda()
    phi_buf = torch.empty((X.shape[0], e.n_features), dtype=torch.float64, device="cuda")

    def loss(v):
        e.shap_values(X, "fp64", leaf_values=v, out=phi_buf)
        return float(((phi_buf - target) ** 2).sum())

    phi0 = e.shap_values(X, "fp64", leaf_values=v0)
    grad = e.shap_backward(X, 2.0 * (phi0 - target), "fp64").cpu().numpy()
    L0 = loss(v0)
    h = 1e-6
    leaves = np.random.default_rng(4).choice(wl.ensemble.n_leaves(), 256, replace=False)
    fd = []
    vp = v0.clone()
    for leaf in leaves:
        vp[leaf] = v0[leaf] + h
        lp = loss(vp)
        vp[leaf] = v0[leaf] - h
        lm = loss(vp)
        vp[leaf] = v0[leaf]
        fd.append((lp - lm) / (2 * h))
    fd = np.array(fd)
    err = np.abs(fd - grad[leaves]).max()
    # rounding of the two loss evaluations: a few hundred ulps of L, over 2h
    tol = 256 * np.finfo(np.float64).eps * L0 / h + 1e-9 * np.abs(grad[leaves]).max()
    print("FD: L=%.4e max|grad|=%.3e max err=%.3e tol=%.3e" % (
        L0, np.abs(grad[leaves]).max(), err, tol), flush=True)
    assert err <= tol


def test_autograd_wrapper(q):
    wl = synth.make_workload("c4_adjoint", T=8, M=200, n_train=5000)
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    target = torch.from_numpy(wl.target).cuda()
    for precision in ("fp32", "fp64"):
        v = torch.from_numpy(wl.ensemble.leaf_values()).cuda().requires_grad_(True)
        phi = q.ShapValues.apply(v, X, e, precision)
        loss = ((phi.double() - target.double()) ** 2).sum()
        loss.backward()
        g_direct = e.shap_backward(X, 2.0 * (phi.detach().double() - target.double()),
                                   precision)
        got, want = v.grad.cpu().numpy(), g_direct.cpu().numpy()
        assert normwise(got, want) <= (1e-6 if precision == "fp32" else 1e-12)


def test_adjoint_edge_cases(q, oracle_mod):
    for seed in range(3):
        rng = np.random.default_rng(500 + seed)
        ens = synth.random_small_ensemble(rng, 5, 6, 6, zero_cover=True)
        X = (np.round(rng.standard_normal((77, 6)) * 2) / 2).astype(np.float32)
        X[::6, 1] = np.nan
        G = rng.normal(size=(77, 6))
        want = oracle_mod.leaf_grad(ens, X, G)
        e = q.Ensemble(ens)
        for precision in ("fp32", "fp64"):
            Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
            g = e.shap_backward(torch.from_numpy(X).cuda(), torch.from_numpy(Gp).cuda(),
                                precision).cpu().numpy()
            assert normwise(g, oracle_mod.leaf_grad(ens, X, Gp)) <= TOL[precision]
    # M = 0: the gradient is zero
    wl = synth.make_workload("c1_small", M=4)
    e = q.Ensemble(wl.ensemble)
    F = wl.ensemble.n_features
    g = e.shap_backward(torch.zeros((0, F), device="cuda"), torch.zeros((0, F), device="cuda"))
    assert g.shape == (wl.ensemble.n_leaves(),) and float(g.abs().max()) == 0.0


@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_adjoint_merged_rows_match_plain(q, oracle_mod, name, over):
    """A merged row gives both of its leaves' gradients from one pass (a
    per-node vector shared by the two leaves); with merging off every leaf
    has its own path.  Both equal the oracle's J^T G."""
    wl = synth.make_workload(name, **over)
    rng = np.random.default_rng(21)
    G = rng.normal(size=wl.X.shape[:1] + (wl.ensemble.n_features,))
    e = q.Ensemble(wl.ensemble)
    assert e.info["n_merged"] > 0
    X = torch.from_numpy(wl.X).cuda()
    want = oracle_mod.leaf_grad(wl.ensemble, wl.X, G)
    for merge in (True, False):
        e.set_sibling_merge(merge)
        g = e.shap_backward(X, torch.from_numpy(G).cuda(), "fp64").cpu().numpy()
        assert normwise(g, want) <= 1e-10, (merge, normwise(g, want))


@pytest.mark.parametrize("M", [1, 77, 700])
def test_adjoint_shared_prefix_walk(q, oracle_mod, M):
    """Rows of at most 8 features reuse the factors (and g_j c_j) of the slots
    they share with the previous row; runs start afresh at chunk boundaries,
    which move with M.  NaN inputs, both tables, both node rules, FP32 and
    FP64 (FP64 with 8 nodes takes the unshared path), against the oracle's
    transposed map."""
    print("case adjoint shared prefix M =", M, flush=True)
    wl = synth.make_workload("c2_values", T=25, M=M, n_train=20000)
    ens = wl.ensemble
    X = wl.X.copy()
    rng = np.random.default_rng(100 + M)
    X[rng.random(X.shape) < 0.05] = np.nan
    G = rng.normal(size=(M, ens.n_features))
    e = q.Ensemble(ens)
    assert e.info["n_value_shared"] > 0
    Xd = torch.from_numpy(X).cuda()
    for precision in ("fp32", "fp64"):
        Gp = G.astype(np.float32).astype(np.float64) if precision == "fp32" else G
        want = oracle_mod.leaf_grad(ens, X, Gp)
        Gd = torch.from_numpy(Gp).cuda()
        if precision == "fp32":
            Gd = Gd.float()
        for merge in (True, False):
            e.set_sibling_merge(merge)
            for policy in ("fixed8", "exact"):
                e.set_node_policy(policy)
                got = e.shap_backward(Xd, Gd, precision).cpu().numpy()
                err = normwise(got, want)
                assert err <= TOL[precision], (precision, merge, policy, err)
