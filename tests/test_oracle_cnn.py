"""Pins of the oracle's parameter-inference network (Sec. 2.3.2-2.3.3)."""

import math

import numpy as np
import torch

import synth
from oracle import cnn


def conv_brute(x, w, b):
    """Seven nested loops, zero padding 1."""
    N, Cin, H, W = x.shape
    Cout = w.shape[0]
    out = np.zeros((N, Cout, H, W))
    for n in range(N):
        for o in range(Cout):
            for i in range(H):
                for j in range(W):
                    acc = b[o]
                    for c in range(Cin):
                        for di in range(3):
                            for dj in range(3):
                                p, q = i + di - 1, j + dj - 1
                                if 0 <= p < H and 0 <= q < W:
                                    acc += w[o, c, di, dj] * x[n, c, p, q]
                    out[n, o, i, j] = acc
    return out


def test_conv_vs_seven_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.max(np.abs(cnn.conv3x3(x, w, b) - conv_brute(x, w, b))) < 1e-12


def test_forward_vs_torch_float64():
    """Independent library: torch's float64 conv2d / linear on the CPU."""
    wts = synth.cnn_weights(seed=3, leaky_alpha=0.01)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 16, 64)) * 2.0
    raw = cnn.forward_raw(x, wts)
    t = torch.from_numpy(x[:, None]).double()
    F = torch.nn.functional
    for l in range(1, 5):
        t = F.conv2d(t, torch.from_numpy(wts[f"conv{l}.w"]).double(),
                     torch.from_numpy(wts[f"conv{l}.b"]).double(), padding=1)
        t = F.leaky_relu(t, 0.01)
    t = F.leaky_relu(F.linear(t.flatten(1), torch.from_numpy(wts["fc1.w"]).double(),
                              torch.from_numpy(wts["fc1.b"]).double()), 0.01)
    t = F.linear(t, torch.from_numpy(wts["fc2.w"]).double(), torch.from_numpy(wts["fc2.b"]).double())
    ref = t.numpy()
    assert np.max(np.abs(raw - ref)) < 1e-10 * max(1.0, np.abs(ref).max())


def test_head_cholesky():
    raw = np.zeros((1, 14))
    raw[0, :4] = [1, 2, 3, 4]
    raw[0, 4:] = np.arange(10) - 5.0
    mu, L = cnn.head(raw)
    assert list(mu[0]) == [1, 2, 3, 4]
    for n, d in enumerate(cnn.DIAG):
        z = raw[0, 4 + d]
        assert abs(L[0, d] - math.log1p(math.exp(z))) < 1e-15
    assert abs(cnn.softplus(np.array([0.0]))[0] - math.log(2.0)) < 1e-16
    Lm = cnn.unpack_L(L[0])
    assert np.all(np.diag(Lm) > 0) and np.allclose(Lm, np.tril(Lm))
    Sig = Lm @ Lm.T
    assert np.all(np.linalg.eigvalsh(Sig) > 0)
    assert Lm[2, 1] == raw[0, 4 + 4]   # row-major packing: L00 L10 L11 L20 L21 ...
