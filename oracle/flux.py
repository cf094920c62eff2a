"""Flux measurement, backward fill and dynamic spectra (Sec. 2.2, Fig. 3).

The flux of a source in a band is the maximum pixel value within a box
around the source's peak position (no Gaussian fitting).  Every measured
source is measured in every band at each step; a newly detected source is
also measured on up to ``t_bf`` cached earlier steps ("backward fill").
Readings: the box is (2 k_flux + 1)^2 intersected with the image, taken on
the quality-controlled cube (a discarded band is all zeros, so its flux is 0
and it is flagged invalid); the dynamic spectrum handed to the network is
the ``ring_len`` steps ending at the episode's last measured step, missing
or invalid cells 0, bands placed on rows of a 16-row grid.
"""

from __future__ import annotations

import numpy as np


def box_max(img: np.ndarray, i: int, j: int, k: int) -> float:
    H, W = img.shape
    r0, r1 = max(0, i - k), min(H, i + k + 1)
    c0, c1 = max(0, j - k), min(W, j + k + 1)
    return float(np.asarray(img[r0:r1, c0:c1], dtype=np.float64).max())


def annulus_mean(img: np.ndarray, i: int, j: int, k: int, w: int) -> float:
    """Mean of the pixels at Chebyshev distance k+1 .. k+w from (i, j) inside
    the image (float64 sum)."""
    H, W = img.shape
    r0, r1 = max(0, i - k - w), min(H, i + k + w + 1)
    c0, c1 = max(0, j - k - w), min(W, j + k + w + 1)
    tot, n = 0.0, 0
    for r in range(r0, r1):
        for c in range(c0, c1):
            if max(abs(r - i), abs(c - j)) > k:
                tot += float(img[r, c])
                n += 1
    return tot / n if n else 0.0


def measure(cube: np.ndarray, i: int, j: int, k: int, bg_width: int = 0) -> np.ndarray:
    """Per-band box maxima at (i, j), float64 [B].  With bg_width > 0 the
    background-subtracted flux: the box maximum minus the mean of the
    surrounding annulus bg_width pixels wide, rounded once to float32."""
    if bg_width <= 0:
        return np.array([box_max(cube[b], i, j, k) for b in range(cube.shape[0])])
    return np.array([float(np.float32(box_max(cube[b], i, j, k) - annulus_mean(cube[b], i, j, k, bg_width)))
                     for b in range(cube.shape[0])])


def window(series: dict, t_end: int, B: int, ring_len: int, grid_rows) -> tuple:
    """Dynamic spectrum [16][ring_len] (float64) and validity [B][ring_len].

    ``series`` maps step -> (flux[B], valid[B] bools)."""
    grid = np.zeros((16, ring_len), dtype=np.float64)
    valid = np.zeros((B, ring_len), dtype=bool)
    for c in range(ring_len):
        tau = t_end - ring_len + 1 + c
        if tau not in series:
            continue
        f, v = series[tau]
        for b in range(B):
            if v[b]:
                grid[grid_rows[b], c] = f[b]
                valid[b, c] = True
    return grid, valid
