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


def measure(cube: np.ndarray, i: int, j: int, k: int) -> np.ndarray:
    """Per-band box maxima at (i, j), float64 [B]."""
    return np.array([box_max(cube[b], i, j, k) for b in range(cube.shape[0])])


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
