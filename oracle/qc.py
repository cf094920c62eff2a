"""Quality control of an image cube (App. A).

Band test: b = per-band mean over all D^2 pixels; z = (b - median b) / MAD(b);
a band whose |z| exceeds the threshold is discarded by imputing zeros.
Readings: MAD is the *median* absolute deviation about the median, without a
consistency factor (the paper says "mean" but cites the median statistic and
asks for robust statistics); when MAD = 0, z = 0 for bands equal to the
median and +inf otherwise.  The same test is also run on the per-band RMS,
which catches the spatially global "whole band noisier" corruption mode the
appendix describes (a band mean cannot).  A band containing any non-finite
pixel is discarded outright and left out of the medians.

Pixel test: zeta = (x - xbar) / s from running per-pixel statistics of the
stream; a band with any |zeta| above the threshold is discarded.  Readings:
cumulative Welford mean / M2 with sample variance (n - 1); the score uses
the statistics of previously *accepted* frames only (corrupt data must not
enter them); the test arms once a band has ``warmup`` accepted frames; only
sky pixels with s > 0 are scored.
"""

from __future__ import annotations

import numpy as np


def band_stats(cube: np.ndarray):
    """Per band: (mean, rms, number of non-finite pixels), float64 sums."""
    B = cube.shape[0]
    x = np.asarray(cube, dtype=np.float64).reshape(B, -1)
    n = x.shape[1]
    finite = np.isfinite(x)
    nonfinite = (~finite).sum(axis=1)
    with np.errstate(invalid="ignore", over="ignore"):
        mean = x.sum(axis=1) / n
        rms = np.sqrt((x * x).sum(axis=1) / n)
    return mean, rms, nonfinite


def robust_z(v: np.ndarray, use: np.ndarray, floor_rel: float = 0.0) -> np.ndarray:
    """(v - median) / max(MAD, floor_rel |median|) over the entries flagged in
    ``use``; others get 0."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros_like(v)
    if not use.any():
        return z
    sel = v[use]
    med = np.median(sel)
    mad = max(np.median(np.abs(sel - med)), floor_rel * abs(med))
    for b in np.nonzero(use)[0]:
        d = v[b] - med
        if mad > 0.0:
            z[b] = d / mad
        else:
            z[b] = 0.0 if d == 0.0 else np.inf
    return z


def band_reject(cube: np.ndarray, band_z: float, rms_z: float, rms_floor: float = 0.05):
    """Bitmask of bands rejected by the non-finite, mean and RMS tests.

    Returns (mask_bits, mean, rms, z_mean, z_rms)."""
    mean, rms, nonfinite = band_stats(cube)
    ok = nonfinite == 0
    zm = robust_z(mean, ok)
    zr = robust_z(rms, ok, rms_floor) if rms_z > 0 else np.zeros_like(zm)
    rej = 0
    for b in range(cube.shape[0]):
        bad = (not ok[b]) or abs(zm[b]) > band_z or (rms_z > 0 and abs(zr[b]) > rms_z)
        if bad:
            rej |= 1 << b
    return rej, mean, rms, zm, zr


class RunningStats:
    """Per-(band, pixel) Welford state of accepted frames."""

    def __init__(self, B: int, H: int, W: int):
        self.n = np.zeros(B, dtype=np.int64)
        self.mean = np.zeros((B, H, W), dtype=np.float64)
        self.m2 = np.zeros((B, H, W), dtype=np.float64)

    def zeta_max(self, b: int, x: np.ndarray, M: np.ndarray, warmup: int) -> float:
        """max |zeta| over sky pixels with s > 0 (0 before warm-up)."""
        n = self.n[b]
        if n < max(warmup, 2):
            return 0.0
        sd = np.sqrt(self.m2[b] / (n - 1))
        use = M & (sd > 0.0)
        if not use.any():
            return 0.0
        with np.errstate(invalid="ignore", over="ignore"):
            z = np.abs(np.asarray(x, dtype=np.float64)[use] - self.mean[b][use]) / sd[use]
        if not np.all(np.isfinite(z)):
            return np.inf
        return float(z.max())

    def update(self, b: int, x: np.ndarray):
        """Welford: n += 1; d = x - mean; mean += d / n; M2 += d (x - mean)."""
        x = np.asarray(x, dtype=np.float64)
        self.n[b] += 1
        d = x - self.mean[b]
        self.mean[b] += d / self.n[b]
        self.m2[b] += d * (x - self.mean[b])
