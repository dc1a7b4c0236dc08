"""qts_shap_values_noalloc (the allocation-free variant of qts_shap_values,
whose scratch is a fixed device array of the library) against
qts_shap_values, called through the C-ABI: two calls in a row with the second
on fewer samples, both precisions, the accumulating and the direct-write
launch forms, leaf-value overrides, and the rejection of a call whose scratch
exceeds the array."""
import ctypes

import numpy as np
import pytest

import synth
from tests.parity import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PREC = {"fp32": 0, "fp64": 1}


def _noalloc(q, e, X, precision, out, leaf=None):
    L = q._lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.qts_shap_values_noalloc(e._h, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                     X.stride(0), ctypes.c_void_p(0 if leaf is None
                                                                  else leaf.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), PREC[precision], s)


@pytest.mark.parametrize("name,over,M2", [
    ("c2_values", dict(T=40, M=700, n_train=20000), 130),   # accumulating launches
    ("c5_deep", dict(T=3, M=300, n_train=30000), 65),       # several buckets
    ("c1_small", dict(M=500), 17),                          # direct writes
])
def test_noalloc_matches_values(name, over, M2):
    import paper_2605_04497_amd as q
    print("case noalloc", name, over, flush=True)
    wl = synth.make_workload(name, **over)
    e = q.Ensemble(wl.ensemble)
    X = torch.from_numpy(wl.X).cuda()
    lv = torch.from_numpy(np.random.default_rng(2).standard_normal(e.n_leaves)).cuda()
    for precision, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        for Xc, leaf in ((X, None), (X[:M2], lv)):   # the second call is smaller
            ref = e.shap_values(Xc, precision, leaf_values=leaf)
            out = torch.full_like(ref, float("nan"))
            rc = _noalloc(q, e, Xc, precision, out, leaf)
            assert rc == 0, q._lib.lib().qts_last_error()
            torch.cuda.synchronize()
            assert bool(torch.isfinite(out).all())
            check(out.double().cpu().numpy(), ref.double().cpu().numpy(), precision,
                  "noalloc %s M=%d" % (name, Xc.shape[0]))
    e.close()


def test_noalloc_rejects_oversize_calls():
    import paper_2605_04497_amd as q
    wl = synth.make_workload("c2_values", T=4, M=8, n_train=20000)
    e = q.Ensemble(wl.ensemble)
    # FP32 with 100 features: 800 bytes of accumulator per sample, beyond the
    # 64 MiB array at 90,000 samples
    X = torch.zeros((90000, e.n_features), device="cuda")
    out = torch.empty((90000, e.n_features), device="cuda")
    rc = _noalloc(q, e, X, "fp32", out)
    assert rc == -3
    assert b"scratch" in q._lib.lib().qts_last_error()
    # a small call still works afterwards
    Xs = torch.from_numpy(wl.X).cuda()
    ref = e.shap_values(Xs, "fp32")
    out = torch.empty_like(ref)
    assert _noalloc(q, e, Xs, "fp32", out) == 0
    torch.cuda.synchronize()
    check(out.double().cpu().numpy(), ref.double().cpu().numpy(), "fp32", "noalloc after reject")
    e.close()
