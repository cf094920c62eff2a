"""Sigma thresholding with clip iterations and peak localisation
(Sec. 2.1.1 Peak Detection, Sec. 2.1.2 Peak Localization, App. C).

Per band image X (already quality-controlled):
  W_i   = M and not Y_{i-1}                       (M: sky mask, Y_0 = 0)
  C, S  = masked normalised estimates with weights W_i
  Y_i   = Y_{i-1} or (M and G*W_i > 0 and x > c + kappa sqrt(s))
  stop when Y_i = Y_{i-1} or after n_iter iterations.
Reading: pixels already above threshold are left out of the next
iteration's statistics ("we clip values"), and the mask accumulates.

Peaks: q_nm = 1 iff x_nm equals the maximum of x over the (2k+1)^2 window
(k = 3) restricted to the image and the sky mask, and (n, m) is in the mask;
ties make every tied pixel a peak.  p = q and y.
"""

from __future__ import annotations

import numpy as np

from .filters import centre_spread


def sigma_clip(X: np.ndarray, M: np.ndarray, g: np.ndarray, kappa: float, n_iter: int,
               trace: list = None):
    """Returns (Y, C, S, den, iterations_run); C, S, den from the last iteration.

    trace (optional list): receives (Y_before, C, S, den) of every iteration
    run, for inspection; it does not change the result."""
    X = np.asarray(X, dtype=np.float64)
    M = np.asarray(M, dtype=bool)
    Y = np.zeros(X.shape, dtype=bool)
    C = S = den = None
    it = 0
    for it in range(1, max(1, n_iter) + 1):
        Wt = M & ~Y
        C, S, den = centre_spread(X, Wt, g)
        if trace is not None:
            trace.append((Y, C, S, den))
        Ynew = Y | (M & (den > 0.0) & (X > C + kappa * np.sqrt(S)))
        changed = bool((Ynew != Y).any())
        Y = Ynew
        if not changed:
            break
    return Y, C, S, den, it


def local_max(X: np.ndarray, M: np.ndarray, k: int) -> np.ndarray:
    """Q: pixel equals the max over its window intersected with image and mask."""
    X = np.asarray(X, dtype=np.float64)
    M = np.asarray(M, dtype=bool)
    H, W = X.shape
    pad = np.full((H + 2 * k, W + 2 * k), -np.inf)
    pad[k:k + H, k:k + W] = np.where(M, X, -np.inf)
    mx = np.full((H, W), -np.inf)
    for di in range(2 * k + 1):
        for dj in range(2 * k + 1):
            np.maximum(mx, pad[di:di + H, dj:dj + W], out=mx)
    return M & (X == mx)


def band_peaks(b: int, X: np.ndarray, M: np.ndarray, g: np.ndarray, kappa: float,
               n_iter: int, k_peak: int):
    """Peak records of one band, in row-major (i, j) order.

    Each record is (b, i, j, x, c, s, sig) with sig = (x - c) / sqrt(s)
    (+inf when s = 0).  Also returns Y, C, S for inspection.
    """
    Y, C, S, den, _ = sigma_clip(X, M, g, kappa, n_iter)
    Q = local_max(X, M, k_peak)
    P = Q & Y
    ii, jj = np.nonzero(P)
    X64 = np.asarray(X, dtype=np.float64)
    recs = []
    for i, j in zip(ii.tolist(), jj.tolist()):
        x, c, s = X64[i, j], C[i, j], S[i, j]
        sig = (x - c) / np.sqrt(s) if s > 0.0 else np.inf
        recs.append((b, i, j, float(x), float(c), float(s), float(sig)))
    return recs, Y, C, S
