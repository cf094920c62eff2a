"""Seeded single-band all-sky images for the source-finder accuracy sweep
(Sec. 3.1 and App. D).  Generation only: no arithmetic of the method.

Recipe (stand-ins for the paper's simulator, whose extended-emission map is
not available):

* point-source fluxes from an exponential distribution whose mean makes
  about 40 % of them fainter than the noise (SNR < 1): P(F < 1) =
  1 - exp(-1 / m) = 0.4, m = -1 / ln(0.6) = 1.958 noise units;
* positions uniform in the circle of diameter D (the sky mask);
* a point-spread function made of a Gaussian main beam (FWHM 3 px) and a few
  random side-lobes, each a Gaussian ridge at radius R_l spanning 0.2 pi rad
  of position angle, normalised to a peak of one;
* standard Gaussian noise plus a smooth inhomogeneous background: a sum of a
  few broad Gaussian blobs (galactic foreground and calibration remnants) so
  that noise and background are not uniform across the image;
* the truth kept per source: position, flux, and SNR = peak flux / noise.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from .sky import SIGMA_PSF, sky_mask

FLUX_MEAN = -1.0 / math.log(0.6)   # P(flux < 1) = 0.4


@dataclasses.dataclass
class SkyTruth:
    rows: np.ndarray
    cols: np.ndarray
    flux: np.ndarray        # peak value of each source (noise sigma = 1)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([int(k) for k in key])))


def random_psf(seed: int, half: int = 15, n_lobes: int = 4) -> np.ndarray:
    """[2 half + 1]^2 PSF: Gaussian main beam plus n_lobes side-lobe arcs of
    0.2 pi rad each, peak 1."""
    g = _rng(seed, 7_000_007)
    u = np.arange(-half, half + 1, dtype=np.float64)
    yy, xx = np.meshgrid(u, u, indexing="ij")
    r = np.hypot(yy, xx)
    th = np.arctan2(yy, xx)
    psf = np.exp(-(r * r) / (2.0 * SIGMA_PSF ** 2))
    for _ in range(n_lobes):
        R = g.uniform(4.0, half - 2.0)
        a = g.uniform(0.05, 0.2)
        th0 = g.uniform(-math.pi, math.pi)
        dth = np.angle(np.exp(1j * (th - th0)))      # wrapped to (-pi, pi]
        arc = (dth >= 0.0) & (dth <= 0.2 * math.pi)
        psf += a * np.exp(-((r - R) ** 2) / (2.0 * 1.0 ** 2)) * arc
    return psf / psf[half, half]


def background(seed: int, H: int, W: int, n_blobs: int = 6) -> np.ndarray:
    g = _rng(seed, 7_000_008)
    ii = np.arange(H)[:, None] + 0.5
    jj = np.arange(W)[None, :] + 0.5
    bg = np.zeros((H, W))
    for _ in range(n_blobs):
        ci, cj = g.uniform(0, H), g.uniform(0, W)
        w = g.uniform(0.05, 0.25) * min(H, W)
        amp = g.uniform(0.5, 3.0)
        bg += amp * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * w * w))
    return bg


def sky_image(seed: int, k: int, D: int = 1024, n_sources: int = 2000, psf_half: int = 15):
    """Image k of a sweep: float32 [D][D] (sky mask applied) and its truth."""
    g = _rng(seed, k, 7_000_009)
    mask = sky_mask(D, D)
    rad = D / 2.0 - 2 * psf_half
    rr = rad * np.sqrt(g.uniform(size=n_sources))
    th = g.uniform(0.0, 2.0 * math.pi, n_sources)
    rows = np.floor(D / 2.0 - 0.5 + rr * np.sin(th) + 0.5).astype(int)
    cols = np.floor(D / 2.0 - 0.5 + rr * np.cos(th) + 0.5).astype(int)
    flux = g.exponential(FLUX_MEAN, n_sources)
    img = g.standard_normal((D, D)) + background(seed + k, D, D)
    psf = random_psf(seed + k, psf_half)
    for r, c, f in zip(rows, cols, flux):
        img[r - psf_half:r + psf_half + 1, c - psf_half:c + psf_half + 1] += f * psf
    img *= mask
    return img.astype(np.float32), SkyTruth(rows, cols, flux), mask


def sweep_images(seed: int, n: int, D: int = 1024, n_sources: int = 2000) -> List[tuple]:
    return [sky_image(seed, k, D, n_sources) for k in range(n)]
