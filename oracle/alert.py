"""Candidate selection on inferred physical parameters and saved candidate
data (Sec. 1, Sec. 2.3.1, Sec. 3.3-3.4).

The network gives per candidate the mean mu = (DM, width, amplitude,
arrival) and the Cholesky factor L of the covariance, Sigma = L L^T
(Sec. 2.3.3); L is packed row by row (L00, L10, L11, L20, ...).  The
standard deviation of the dispersion measure is sqrt(Sigma_00).  Low
dispersion measures are excluded (Sec. 2.3.1: nearby noise is not
dispersed); on real data the paper keeps inferred DM above 50 and ranks the
candidates by sigma_DM (Sec. 3.4), and reads sigma_DM above 50 as the false-
positive mode (Sec. 3.3).  Test infrastructure: plain numpy, float64.
"""

from __future__ import annotations

import numpy as np


def unpack_cholesky(Lp: np.ndarray) -> np.ndarray:
    """[n][10] packed row-major lower triangle -> [n][4][4]."""
    Lp = np.asarray(Lp, dtype=np.float64)
    out = np.zeros((Lp.shape[0], 4, 4))
    k = 0
    for i in range(4):
        for j in range(i + 1):
            out[:, i, j] = Lp[:, k]
            k += 1
    return out


def sigma_dm(Lp: np.ndarray) -> np.ndarray:
    """sqrt(Sigma_00) of Sigma = L L^T for each row."""
    Lm = unpack_cholesky(Lp)
    Sigma = Lm @ np.transpose(Lm, (0, 2, 1))
    return np.sqrt(Sigma[:, 0, 0])


def select(mu: np.ndarray, Lp: np.ndarray, dm_min: float = 50.0, sigma_max: float = 50.0):
    """Row indices with mu_DM > dm_min and sigma_DM <= sigma_max, ordered by
    sigma_DM ascending, ties by row (values compared as given)."""
    mu = np.asarray(mu, dtype=np.float64)
    sg = sigma_dm(Lp)
    keep = [i for i in range(len(mu)) if mu[i, 0] > dm_min and sg[i] <= sigma_max]
    return sorted(keep, key=lambda i: (sg[i], i)), sg


def cutouts(cache: dict, rejected: dict, row: int, col: int, half: int, t_first: int, n_steps: int, B: int,
            H: int, W: int):
    """[n_steps][B][2h+1][2h+1] boxes of the cached quality-controlled images
    (zero outside the image and for steps no longer cached), and the cached
    flags."""
    side = 2 * half + 1
    out = np.zeros((n_steps, B, side, side), dtype=np.float32)
    have = np.zeros(n_steps, dtype=bool)
    for k in range(n_steps):
        tau = t_first + k
        if tau not in cache:
            continue
        have[k] = True
        for di in range(-half, half + 1):
            for dj in range(-half, half + 1):
                i, j = row + di, col + dj
                if 0 <= i < H and 0 <= j < W:
                    out[k, :, di + half, dj + half] = cache[tau][:, i, j]
    return out, have
