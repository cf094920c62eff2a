"""Parameter-inference network and Gaussian head (Sec. 2.3.2-2.3.3).

A hidden unit is phi(x.w + b) with the leaky rectifier phi(h) = h for h >= 0
and alpha h otherwise (alpha = 0 gives the plain rectifier); the last layer
is linear.  The network maps a dynamic spectrum to [mu ; L], where L is a
lower-triangular matrix with positive diagonal (a Cholesky factor, so
Sigma = L L^T is a valid covariance).

Architecture (the paper gives none; these are the sizes the network kernels
serve): input 1 x 16 x 64; four 3x3 convolutions, stride 1, zero padding 1,
1->32->32->64->64 channels, each followed by phi; flatten in (channel, row,
column) order; dense 65536->128 with phi; dense 128->14.  Outputs 0..3 are
mu (DM, width, amplitude, arrival); outputs 4..13 fill L row by row
(L00, L10, L11, L20, L21, L22, L30, L31, L32, L33); the diagonal passes
through softplus(z) = log(1 + e^z) to make it positive.

Evaluated in float64 with im2col + matmul.
"""

from __future__ import annotations

import numpy as np

DIAG = (0, 2, 5, 9)   # positions of L00, L11, L22, L33 in the packed 10


def act(h: np.ndarray, alpha: float) -> np.ndarray:
    return np.where(h >= 0.0, h, alpha * h)


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [N][Cin][H][W], w [Cout][Cin][3][3] -> [N][Cout][H][W] (correlation, pad 1)."""
    N, Cin, H, W = x.shape
    Cout = w.shape[0]
    pad = np.zeros((N, Cin, H + 2, W + 2), dtype=np.float64)
    pad[:, :, 1:H + 1, 1:W + 1] = x
    cols = np.empty((N, H, W, Cin, 3, 3), dtype=np.float64)
    for di in range(3):
        for dj in range(3):
            cols[..., di, dj] = pad[:, :, di:di + H, dj:dj + W].transpose(0, 2, 3, 1)
    out = cols.reshape(N * H * W, Cin * 9) @ np.asarray(w, np.float64).reshape(Cout, Cin * 9).T
    out += np.asarray(b, np.float64)[None, :]
    return out.reshape(N, H, W, Cout).transpose(0, 3, 1, 2)


def softplus(z: np.ndarray) -> np.ndarray:
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def forward_raw(x: np.ndarray, wts: dict) -> np.ndarray:
    """x [N][16][64] (or [N][1][16][64]) -> raw outputs [N][14], float64."""
    a = np.asarray(x, dtype=np.float64)
    if a.ndim == 3:
        a = a[:, None]
    alpha = float(wts.get("alpha", 0.0))
    for l in range(1, 5):
        a = act(conv3x3(a, wts[f"conv{l}.w"], wts[f"conv{l}.b"]), alpha)
    h = a.reshape(a.shape[0], -1)
    h = act(h @ np.asarray(wts["fc1.w"], np.float64).T + np.asarray(wts["fc1.b"], np.float64), alpha)
    return h @ np.asarray(wts["fc2.w"], np.float64).T + np.asarray(wts["fc2.b"], np.float64)


def head(raw: np.ndarray):
    """raw [N][14] -> (mu [N][4], L packed [N][10]) with softplus diagonal."""
    mu = raw[:, :4].copy()
    L = raw[:, 4:14].copy()
    for d in DIAG:
        L[:, d] = softplus(L[:, d])
    return mu, L


def forward(x: np.ndarray, wts: dict):
    return head(forward_raw(x, wts))


def unpack_L(Lp: np.ndarray) -> np.ndarray:
    """Packed row-major lower triangle [10] -> 4x4 matrix."""
    L = np.zeros((4, 4))
    n = 0
    for r in range(4):
        for c in range(r + 1):
            L[r, c] = Lp[n]
            n += 1
    return L
