"""The allocation-free network entry point (lpf_infer_windows_static): its
intermediate buffers live in the library's static device array instead of
the model's workspace.  Checked through the C ABI against the workspace
form lpf_infer_windows on the same windows (the same kernels and summation
order, so bitwise equal) and, for float32, against the FP64 oracle at the
parity tolerance (1e-5 of the condition scale); two calls in a row, the
second with fewer windows, so stale contents of the array cannot leak into
a result."""

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn

from parity import cnn_scale

pytestmark = pytest.mark.gpu


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("prec", [0, 1])
def test_static_inference_matches_workspace_form(prec):
    torch = _torch_cuda()
    from paper_2103_15418_amd import Model
    wts = synth.cnn_weights(seed=7)
    model = Model(wts, precision=prec, max_batch=64)
    rng = np.random.default_rng(2024 + prec)
    for n in (32, 5):
        print(f"static inference prec={prec} n={n}", flush=True)
        x = (rng.standard_normal((n, 16, 64)) * 2.0).astype(np.float32)
        xd = torch.from_numpy(x).cuda()
        mu_ref, L_ref = model.infer_windows(xd)
        mu = torch.full((n, 4), float("nan"), device="cuda")
        L = torch.full((n, 10), float("nan"), device="cuda")
        torch.cuda.synchronize()
        assert model.infer_windows_static(xd, mu, L) == 0
        torch.cuda.synchronize()
        mu_h, L_h = mu.cpu().numpy(), L.cpu().numpy()
        assert np.array_equal(mu_h, mu_ref.cpu().numpy()), (prec, n)
        assert np.array_equal(L_h, L_ref.cpu().numpy()), (prec, n)
        if prec == 0:
            mo, Lo = ocnn.forward(x.astype(np.float64), wts)
            sc = cnn_scale(x.astype(np.float64), wts)
            assert np.all(np.abs(mu_h - mo) <= 1e-5 * sc[:, :4] + 1e-6), n
            assert np.all(np.abs(L_h - Lo) <= 1e-5 * sc[:, 4:] + 1e-6), n


def test_static_inference_rejects_oversized_batch():
    torch = _torch_cuda()
    from paper_2103_15418_amd import Model
    from paper_2103_15418_amd._abi import LPF_EINVAL
    model = Model(synth.cnn_weights(seed=7), max_batch=64)
    x = torch.zeros((33, 16, 64), device="cuda")
    mu = torch.zeros((33, 4), device="cuda")
    L = torch.zeros((33, 10), device="cuda")
    assert model.infer_windows_static(x, mu, L) == LPF_EINVAL
    assert model.infer_windows_static(x[:0], mu[:0], L[:0]) == 0
