"""Kernels and the local centre / spread estimates (Sec. 2.1.1, Peak Detection).

The paper defines the Gaussian kernel
    G(n, m, s) = exp(-(n^2 + m^2) / (2 s^2)) / Z
with Z the sum of the same exponential over the kernel's support, and the
estimates
    C = G * X,      S = G * (X - C)^2     (square taken per pixel).

Readings used here (the paper is silent on them):
* the support is the square [-k, k]^2 with k = ceil(3 s) (the normaliser is
  the sum over the kernel's own support, so G sums to one);
* "*" is 2-D correlation with zero extension outside the image, applied to
  the masked data W.X and normalised by G*W ("normalised convolution"), so
  that image edges and the circular sky mask do not bias C and S towards
  zero:  C = (G*(W.X)) / (G*W),  S = (G*(W.(X-C)^2)) / (G*W), both 0 where
  G*W = 0;
* the uniform alternatives the paper mentions are the square box
  1/(2k+1)^2 and the circular (disk) kernel, uniform on the offsets with
  u^2 + v^2 <= k^2; the disk is not separable and is applied as a 2-D sum.

Because exp(-(n^2+m^2)/2s^2) = exp(-n^2/2s^2) exp(-m^2/2s^2), G equals the
outer product g (x) g of the 1-D taps g_u = exp(-u^2/2s^2) / sum_v exp(-v^2/2s^2)
exactly (and Z = Z_1^2); the 2-D correlation is therefore evaluated as a row
correlation followed by a column correlation.  The brute-force 2-D sum in the
tests pins this.
"""

from __future__ import annotations

import numpy as np

from .config import KERNEL_BOX, KERNEL_DISK, KERNEL_GAUSS


def taps_1d(kernel: int, s: float, k: int) -> np.ndarray:
    """float64 taps g_u, u = -k..k, summing to one."""
    u = np.arange(-k, k + 1, dtype=np.float64)
    if kernel == KERNEL_GAUSS:
        e = np.exp(-(u * u) / (2.0 * s * s))
    elif kernel == KERNEL_BOX:
        e = np.ones_like(u)
    else:
        raise ValueError("unknown kernel")
    return e / e.sum()


def disk_kernel(k: int) -> np.ndarray:
    """float64 [2k+1][2k+1]: 1/N on the offsets with u^2 + v^2 <= k^2."""
    u = np.arange(-k, k + 1)
    inside = (u[:, None] ** 2 + u[None, :] ** 2) <= k * k
    return inside / inside.sum()


def kernel_taps(kernel: int, s: float, k: int) -> np.ndarray:
    """1-D taps of a separable kernel, or the 2-D disk kernel."""
    if kernel == KERNEL_DISK:
        return disk_kernel(k)
    return taps_1d(kernel, s, k)


def correlate_kernel2d(img: np.ndarray, K: np.ndarray) -> np.ndarray:
    """out[i, j] = sum_{u,v} K[u, v] img[i+u, j+v], zero outside the image."""
    k = (K.shape[0] - 1) // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * k, W + 2 * k), dtype=np.float64)
    pad[k:k + H, k:k + W] = img
    out = np.zeros((H, W), dtype=np.float64)
    for a in range(2 * k + 1):
        for b in range(2 * k + 1):
            if K[a, b] != 0.0:
                out += K[a, b] * pad[a:a + H, b:b + W]
    return out


def correlate_rows(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """out[i, j] = sum_u g[u] img[i, j+u], zero outside the image."""
    k = (len(g) - 1) // 2
    H, W = img.shape
    pad = np.zeros((H, W + 2 * k), dtype=np.float64)
    pad[:, k:k + W] = img
    out = np.zeros((H, W), dtype=np.float64)
    for t in range(2 * k + 1):
        out += g[t] * pad[:, t:t + W]
    return out


def correlate_cols(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """out[i, j] = sum_u g[u] img[i+u, j], zero outside the image."""
    return correlate_rows(img.T, g).T


def correlate_2d(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """(g (x) g) correlated with img, zero extension (g 1-D taps), or the 2-D
    kernel g correlated with img."""
    if np.ndim(g) == 2:
        return correlate_kernel2d(np.asarray(img, dtype=np.float64), g)
    return correlate_cols(correlate_rows(np.asarray(img, dtype=np.float64), g), g)


def centre_spread(X: np.ndarray, Wt: np.ndarray, g: np.ndarray):
    """Masked, normalised centre and spread of one band image.

    X  : float image (any float dtype; evaluated in float64)
    Wt : bool/0-1 weight plane (sky mask and not already clipped)
    g  : 1-D taps of a separable kernel, or a 2-D kernel
    Returns (C, S, den) in float64.
    """
    X = np.asarray(X, dtype=np.float64)
    w = np.asarray(Wt, dtype=np.float64)
    den = correlate_2d(w, g)
    pos = den > 0.0
    safe = np.where(pos, den, 1.0)
    C = np.where(pos, correlate_2d(w * X, g) / safe, 0.0)
    R = X - C
    S = np.where(pos, correlate_2d(w * R * R, g) / safe, 0.0)
    return C, S, den


def prefilter(X: np.ndarray, M: np.ndarray, g_psf: np.ndarray) -> np.ndarray:
    """Image correlated with the PSF taps over the sky mask, normalised like C:
    (G_psf*(M.X)) / (G_psf*M), 0 where the denominator is 0 (the matched
    filter of a point source in white noise)."""
    C, _, _ = centre_spread(X, M, g_psf)
    return C
