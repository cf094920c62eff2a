"""Pins of the detection variants of the oracle: circular uniform kernel
(Sec. 2.1.1), matched PSF pre-filter, background-subtracted flux."""

import math
import os

import numpy as np
import pytest

from oracle.config import KERNEL_DISK, OracleConfig
from oracle.detect import sigma_clip
from oracle.filters import centre_spread, disk_kernel, prefilter, taps_1d
from oracle.flux import annulus_mean, box_max, measure
from oracle.pipeline import OracleStream

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_disk_single_hot_pixel():
    X = np.zeros((7, 7), np.float32)
    X[3, 3] = 10.0
    M = np.ones((7, 7), bool)
    K = disk_kernel(1)
    assert (K > 0).sum() == 5
    C, S, _ = centre_spread(X, M, K)
    Y1 = sigma_clip(X, M, K, 1.0, 1)[0]
    Y2 = sigma_clip(X, M, K, 2.0, 1)[0]
    for line in open(os.path.join(GOLDEN, "disk1_single_hot_pixel.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, i, j, v = line.split()
        got = {"C": C, "S": S, "Y1": Y1, "Y2": Y2}[key][int(i), int(j)]
        assert abs(float(got) - float(v)) < 1e-12, (key, i, j)


@pytest.mark.parametrize("seed,k", [(0, 2), (1, 3), (2, 5)])
def test_disk_vs_brute_force(seed, k):
    """Masked normalised disk estimates against a per-pixel loop over the
    offsets with u^2 + v^2 <= k^2."""
    rng = np.random.default_rng(seed)
    H, W = 17, 23
    X = rng.standard_normal((H, W)).astype(np.float32)
    M = rng.uniform(size=(H, W)) > 0.25
    C, S, den = centre_spread(X, M, disk_kernel(k))
    offs = [(u, v) for u in range(-k, k + 1) for v in range(-k, k + 1) if u * u + v * v <= k * k]

    def est(vals):
        out = np.zeros((H, W))
        cnt = np.zeros((H, W))
        for i in range(H):
            for j in range(W):
                for u, v in offs:
                    p, q = i + u, j + v
                    if 0 <= p < H and 0 <= q < W and M[p, q]:
                        out[i, j] += vals[p, q]
                        cnt[i, j] += 1
        return np.where(cnt > 0, out / np.maximum(cnt, 1), 0.0), cnt
    Cb, cnt = est(X.astype(np.float64))
    Sb, _ = est((X.astype(np.float64) - Cb) ** 2)
    assert np.allclose(C, Cb, atol=1e-12, rtol=0) and np.allclose(S, Sb, atol=1e-12, rtol=0)
    assert np.allclose(den * len(offs), cnt, atol=1e-9)


def test_disk_constant_image():
    X = np.full((30, 30), 3.25, np.float32)
    M = np.ones((30, 30), bool)
    M[:, :5] = False
    C, S, den = centre_spread(X, M, disk_kernel(6))
    pos = den > 0
    assert np.allclose(C[pos], 3.25, atol=1e-12) and np.allclose(S[pos], 0.0, atol=1e-12)


def test_prefilter_point_source_closed_form():
    """A noise-free Gaussian PSF of width s_p at an integer centre far from the
    edges: the pre-filtered centre value is A (Z(s_p / sqrt 2) / Z(s_p))^2 with
    Z(s) = sum_u exp(-u^2 / (2 s^2)) over the taps' support (an explicit 2-D
    sum gives the same); a constant image stays constant, also at the mask's
    edge."""
    sp, A, k = 1.274, 7.0, 6
    n = 41
    u = np.arange(n) - 20
    X = (A * np.exp(-(u[:, None] ** 2 + u[None, :] ** 2) / (2 * sp ** 2))).astype(np.float64)
    M = np.ones((n, n), bool)
    g = taps_1d(0, sp, k)
    out = prefilter(X, M, g)
    v = np.arange(-k, k + 1)
    Z = lambda s: np.exp(-(v ** 2) / (2 * s * s)).sum()
    closed = A * (Z(sp / math.sqrt(2)) / Z(sp)) ** 2
    brute = sum(g[a] * g[b] * X[20 + a - k, 20 + b - k] for a in range(2 * k + 1) for b in range(2 * k + 1))
    assert abs(out[20, 20] - closed) < 1e-12 and abs(out[20, 20] - brute) < 1e-12
    Mc = np.zeros((n, n), bool)
    Mc[5:30, 8:35] = True
    const = prefilter(np.full((n, n), 2.5), Mc, g)
    assert np.allclose(const[Mc], 2.5, atol=1e-12)


def test_background_subtracted_flux_hand_case():
    """Box k = 1 around (3,3) holds the maximum 9; the annulus of width 1 (the
    16 pixels at Chebyshev distance 2) holds 1 everywhere except one 5: mean
    (15 + 5) / 16 = 1.25, flux 9 - 1.25 = 7.75.  At a corner the annulus is
    clipped to the image."""
    img = np.zeros((9, 9), np.float32)
    img[1:6, 1:6] = 1.0
    img[2:5, 2:5] = 0.0
    img[3, 4] = 9.0
    img[1, 1] = 5.0
    assert box_max(img, 3, 3, 1) == 9.0
    assert abs(annulus_mean(img, 3, 3, 1, 1) - 1.25) < 1e-15
    assert measure(img[None], 3, 3, 1, 1)[0] == np.float32(7.75)
    # corner (0, 0): box rows/cols 0..1, annulus = Chebyshev 2 inside the image: (0..2, 2) and (2, 0..1)
    ring = [img[r, c] for r in range(0, 3) for c in range(0, 3) if max(r, c) == 2]
    assert abs(annulus_mean(img, 0, 0, 1, 1) - np.mean(ring)) < 1e-15


def test_stream_with_variants_runs():
    """The oracle stream with the disk kernel, the pre-filter and the
    background-subtracted flux finds an injected bright source."""
    rng = np.random.default_rng(5)
    B, H, W = 2, 64, 64
    cfg = OracleConfig(B=B, H=H, W=W, kernel=KERNEL_DISK, k_bg=8, kappa=4.0, prefilter_sigma=1.274,
                       flux_bg_width=2)
    o = OracleStream(cfg)
    assert o.cfg.prefilter_k == 6
    cube = rng.standard_normal((B, H, W)).astype(np.float32)
    cube[:, 30:33, 30:33] += 12.0
    o.ingest(0, cube)
    peaks, new, ended = o.detect()
    assert any(abs(p[1] - 31) <= 1 and abs(p[2] - 31) <= 1 for p in peaks)
    o.extract_flux()
    sid = new[0]
    f, v = o.series[sid][0]
    assert np.all(v) and np.all(f > 5)
