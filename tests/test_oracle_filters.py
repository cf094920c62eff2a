"""Pins of the oracle's kernel and centre/spread estimates (Sec. 2.1.1)."""

import math

import numpy as np
import pytest
from scipy import ndimage

from oracle.config import KERNEL_BOX, KERNEL_GAUSS
from oracle.filters import centre_spread, correlate_2d, taps_1d


def gauss2d_brute(s, k):
    """G(n, m) written from the 2-D definition, Z summed over the 2-D support."""
    G = np.zeros((2 * k + 1, 2 * k + 1))
    for n in range(-k, k + 1):
        for m in range(-k, k + 1):
            G[n + k, m + k] = math.exp(-(n * n + m * m) / (2.0 * s * s))
    return G / G.sum()


def masked_normalised_brute(X, Wt, G):
    """Direct 2-D sums with explicit loops (zero extension)."""
    H, W = X.shape
    k = (G.shape[0] - 1) // 2
    C = np.zeros((H, W))
    S = np.zeros((H, W))
    den = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            num = d = 0.0
            for n in range(-k, k + 1):
                for m in range(-k, k + 1):
                    p, q = i + n, j + m
                    if 0 <= p < H and 0 <= q < W and Wt[p, q]:
                        num += G[n + k, m + k] * X[p, q]
                        d += G[n + k, m + k]
            den[i, j] = d
            C[i, j] = num / d if d > 0 else 0.0
    for i in range(H):
        for j in range(W):
            if den[i, j] <= 0:
                continue
            acc = 0.0
            for n in range(-k, k + 1):
                for m in range(-k, k + 1):
                    p, q = i + n, j + m
                    if 0 <= p < H and 0 <= q < W and Wt[p, q]:
                        acc += G[n + k, m + k] * (X[p, q] - C[p, q]) ** 2
            S[i, j] = acc / den[i, j]
    return C, S, den


@pytest.mark.parametrize("s,k", [(1.0, 3), (2.5, 6), (8.0, 24), (0.7, 1)])
def test_taps_sum_and_separable_equals_2d_definition(s, k):
    g = taps_1d(KERNEL_GAUSS, s, k)
    assert len(g) == 2 * k + 1
    assert abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1], rtol=0, atol=0)
    G = gauss2d_brute(s, k)
    assert np.max(np.abs(np.outer(g, g) - G)) < 1e-15


def test_box_taps():
    g = taps_1d(KERNEL_BOX, 3.0, 2)
    assert np.all(g == 0.2)


@pytest.mark.parametrize("shape,k,s,seed", [((1, 1), 1, 1.0, 0), ((5, 7), 2, 1.3, 1),
                                            ((17, 9), 3, 2.0, 2), ((23, 31), 4, 1.5, 3),
                                            ((40, 40), 6, 2.2, 4), ((12, 40), 6, 3.0, 5)])
def test_centre_spread_vs_brute_force_2d(shape, k, s, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal(shape).astype(np.float32)
    Wt = rng.uniform(size=shape) > 0.3
    g = taps_1d(KERNEL_GAUSS, s, k)
    C, S, den = centre_spread(X, Wt, g)
    Cb, Sb, denb = masked_normalised_brute(X.astype(np.float64), Wt, gauss2d_brute(s, k))
    assert np.max(np.abs(den - denb)) < 1e-12
    scale = max(1.0, np.abs(X).max())
    assert np.max(np.abs(C - Cb)) < 1e-12 * scale
    assert np.max(np.abs(S - Sb)) < 1e-12 * scale ** 2


def test_box_kernel_vs_brute_force():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((19, 21))
    Wt = rng.uniform(size=X.shape) > 0.2
    k = 3
    g = taps_1d(KERNEL_BOX, 0.0, k)
    G = np.full((2 * k + 1, 2 * k + 1), 1.0 / (2 * k + 1) ** 2)
    C, S, den = centre_spread(X, Wt, g)
    Cb, Sb, denb = masked_normalised_brute(X, Wt, G)
    assert np.max(np.abs(C - Cb)) < 1e-12 and np.max(np.abs(S - Sb)) < 1e-12


def test_numerator_denominator_vs_scipy_correlate1d():
    """Independent library: scipy's 1-D correlation with constant (zero) mode."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal((64, 80))
    M = rng.uniform(size=X.shape) > 0.1
    g = taps_1d(KERNEL_GAUSS, 4.0, 12)
    for plane in (M * X, M.astype(np.float64)):
        ref = ndimage.correlate1d(ndimage.correlate1d(plane, g, axis=1, mode="constant"),
                                  g, axis=0, mode="constant")
        assert np.max(np.abs(correlate_2d(plane, g) - ref)) < 1e-13


def test_constant_image_invariant():
    g = taps_1d(KERNEL_GAUSS, 3.0, 9)
    M = np.ones((50, 60), dtype=bool)
    M[:, :5] = False  # masked strip
    X = np.full((50, 60), 2.75)
    C, S, den = centre_spread(X, M, g)
    assert np.max(np.abs(C - 2.75)) < 1e-12
    assert np.max(np.abs(S)) < 1e-12


def test_affine_transpose_shift_invariants():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((48, 48))
    M = rng.uniform(size=X.shape) > 0.15
    g = taps_1d(KERNEL_GAUSS, 2.0, 6)
    C, S, _ = centre_spread(X, M, g)
    a, beta = 3.5, -1.25
    C2, S2, _ = centre_spread(a * X + beta, M, g)
    sel = correlate_2d(M.astype(float), g) > 0
    assert np.max(np.abs(C2[sel] - (a * C[sel] + beta))) < 1e-12
    assert np.max(np.abs(S2[sel] - a * a * S[sel])) < 1e-11
    Ct, St, _ = centre_spread(X.T, M.T, g)
    assert np.max(np.abs(Ct - C.T)) < 1e-13 and np.max(np.abs(St - S.T)) < 1e-13
    # shift by (5, 7) on an unmasked larger image: interior agrees
    Y = rng.standard_normal((80, 80))
    ones = np.ones_like(Y, dtype=bool)
    Ca, Sa, _ = centre_spread(Y, ones, g)
    Cb, Sb, _ = centre_spread(np.roll(np.roll(Y, 5, 0), 7, 1), ones, g)
    inner = (slice(6 + 6 + 5, 80 - 12), slice(6 + 6 + 7, 80 - 12))
    assert np.max(np.abs(np.roll(np.roll(Ca, 5, 0), 7, 1)[inner] - Cb[inner])) < 1e-12
    assert np.max(np.abs(np.roll(np.roll(Sa, 5, 0), 7, 1)[inner] - Sb[inner])) < 1e-12


def test_gaussian_source_centre_closed_form():
    """Noise-free Gaussian source of peak A, width sp: the continuous
    convolution gives C(centre) = A sp^2 / (sp^2 + s^2)."""
    sp = 3.0 / (2 * math.sqrt(2 * math.log(2)))
    s, A, D = 8.0, 10.0, 161
    i = np.arange(D) - D // 2
    X = A * np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2 * sp * sp))
    g = taps_1d(KERNEL_GAUSS, s, 24)
    C, S, _ = centre_spread(X, np.ones_like(X, dtype=bool), g)
    expect = A * sp * sp / (sp * sp + s * s)
    assert abs(C[D // 2, D // 2] - expect) / expect < 1e-2


def test_edge_normalisation_keeps_constants_at_corners():
    g = taps_1d(KERNEL_GAUSS, 8.0, 24)
    X = np.full((30, 30), -4.0)
    C, S, den = centre_spread(X, np.ones_like(X, dtype=bool), g)
    assert abs(C[0, 0] + 4.0) < 1e-12 and abs(S[0, 0]) < 1e-12
    assert 0.2 < den[0, 0] < 0.3   # a quarter of the kernel mass in the image (+ truncation)
