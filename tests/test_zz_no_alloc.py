"""fmm_mlp_grad_noalloc (the selector's training gradient with the library's fixed device
scratch, for callers that cannot allocate) against fmm_mlp_grad, through the C ABI: two
calls in a row, the second with a smaller batch, so leftovers of the first call in the
shared scratch would show; and against the FP64 reference."""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hf = pytest.importorskip("paper_2006_14952_amd")
from paper_2006_14952_amd import learned  # noqa: E402


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, 16)).astype(np.float32) * 2 + 1
    y = rng.integers(0, 8, B).astype(np.int32)
    w = learned.init_params(seed) + rng.standard_normal(5768).astype(np.float32) * 0.01
    mu = rng.standard_normal(16).astype(np.float32) * 0.3
    isd = (0.5 + rng.random(16)).astype(np.float32)
    cw = (0.5 + rng.random(8)).astype(np.float32)
    return X, y, w, mu, isd, cw


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _p(t):
    return C.c_void_p(t.data_ptr())


def _call(name, w, mu, isd, X, y, cw, stream):
    g = torch.full((5768,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    rc = getattr(hf.lib(), name)(_p(w), _p(mu), _p(isd), _p(X), _p(y), _p(cw), int(X.shape[0]), _p(g), _p(loss),
                                 C.c_void_p(stream.cuda_stream))
    assert rc == 0, hf.lib().fmm_last_error().decode()
    stream.synchronize()
    return float(loss.item()), g.cpu().numpy()


def test_noalloc_gradient_equals_the_allocating_entry_point_on_two_calls():
    stream = torch.cuda.Stream()
    for B, seed in ((3000, 21), (777, 22)):  # the second call is smaller than the first
        X, y, w, mu, isd, cw = _batch(B, seed)
        args = [_dev(a) for a in (w, mu, isd, X, y, cw)]
        l_ref, g_ref = _call("fmm_mlp_grad", *args, stream)
        l_na, g_na = _call("fmm_mlp_grad_noalloc", *args, stream)
        assert np.all(np.isfinite(g_na)) and np.isfinite(l_na)
        # the same kernels; the class-weight sum is formed on the device (atomics), so
        # the two agree to FP32 rounding, not bit for bit
        assert abs(l_na - l_ref) <= 1e-5 * abs(l_ref)
        np.testing.assert_allclose(g_na, g_ref, rtol=1e-4, atol=1e-6 * np.abs(g_ref).max())
        l64, g64 = omlp.loss_and_grad(w.astype(np.float64), X, y, cw, mu, isd)
        assert abs(l_na - l64) < 1e-5 * max(1.0, abs(l64))
        np.testing.assert_allclose(g_na, g64, rtol=2e-3, atol=2e-6 * np.abs(g64).max())


def test_noalloc_rejects_batches_beyond_its_scratch():
    X, y, w, mu, isd, cw = _batch(8193, 23)
    args = [_dev(a) for a in (w, mu, isd, X, y, cw)]
    g = torch.zeros(5768, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rc = hf.lib().fmm_mlp_grad_noalloc(*[_p(a) for a in args], 8193, _p(g), _p(loss), None)
    assert rc == hf.FMM_ERR_ARG and "8192" in hf.lib().fmm_last_error().decode()
