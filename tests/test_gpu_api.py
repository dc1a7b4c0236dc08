"""The Python binding rejects output and gradient buffers that do not match
the call (type, shape, layout, device) before the library is called, so no
kernel ever writes through a wrong pointer."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ens():
    import paper_2605_04497_amd as q
    wl = synth.make_workload("c1_small", M=40)
    e = q.Ensemble(wl.ensemble)
    return e, torch.from_numpy(wl.X).cuda()


def _calls_library(monkeypatch):
    """Replace the library handle so any call through it fails the test."""
    import paper_2605_04497_amd._lib as L
    import paper_2605_04497_amd.api as api

    class NoCalls:
        def __getattr__(self, name):
            raise AssertionError("library called: %s" % name)
    monkeypatch.setattr(api.L, "lib", lambda: NoCalls())
    return L


def test_bad_outputs_rejected_before_any_launch(ens, monkeypatch):
    e, X = ens
    M, F = X.shape[0], e.n_features
    bad_values = [
        torch.empty((M, F), dtype=torch.float64, device="cuda"),       # wrong type
        torch.empty((M - 1, F), dtype=torch.float32, device="cuda"),   # short
        torch.empty((F, M), dtype=torch.float32, device="cuda").t(),   # strided
        torch.empty((M, F), dtype=torch.float32),                      # host memory
    ]
    _calls_library(monkeypatch)
    for out in bad_values:
        with pytest.raises((TypeError, ValueError)):
            e.shap_values(X, "fp32", out=out)
    with pytest.raises((TypeError, ValueError)):
        e.shap_values(X, "fp64", out=torch.empty((M, F), dtype=torch.float32, device="cuda"))
    with pytest.raises((TypeError, ValueError)):
        e.shap_interactions(X, "fp32", out=torch.empty((M, F, F - 1), device="cuda"))
    with pytest.raises((TypeError, ValueError)):
        e.shap_interactions(X, "fp32", with_phi=True,
                            out_phi=torch.empty((M, F), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        e.shap_interactions(X, "fp32", out_phi=torch.empty((M, F), device="cuda"))
    T3 = F * (F - 1) * (F - 2) // 6
    with pytest.raises((TypeError, ValueError)):
        e.shap_interactions3(X, "fp32", out=torch.empty((M, T3 + 1), device="cuda"))
    # gradients: host tensor, wrong shape; gradient output of the wrong type
    with pytest.raises(ValueError):
        e.shap_backward(X, torch.zeros((M, F)), "fp32")
    with pytest.raises(ValueError):
        e.shap_backward(X, torch.zeros((M, F + 1), device="cuda"), "fp32")
    with pytest.raises((TypeError, ValueError)):
        e.shap_backward(X, torch.zeros((M, F), device="cuda"), "fp32",
                        out=torch.empty(e.n_leaves, dtype=torch.float32, device="cuda"))
    # leaf values on the host
    with pytest.raises(TypeError):
        e.shap_values(X, "fp32", leaf_values=torch.zeros(e.n_leaves, dtype=torch.float64))


def test_good_outputs_accepted(ens):
    e, X = ens
    M, F = X.shape[0], e.n_features
    out = torch.full((M, F), float("nan"), device="cuda")
    e.shap_values(X, "fp32", out=out)
    ref = e.shap_values(X, "fp32")
    torch.cuda.synchronize()
    assert torch.allclose(out, ref, rtol=1e-6, atol=1e-9)
    Phi = torch.empty((M, F, F), dtype=torch.float64, device="cuda")
    phi = torch.empty((M, F), dtype=torch.float64, device="cuda")
    e.shap_interactions(X, "fp64", with_phi=True, out=Phi, out_phi=phi)
    torch.cuda.synchronize()
    assert np.allclose(phi.cpu().numpy(), Phi.sum(2).cpu().numpy(), rtol=0, atol=1e-12)
