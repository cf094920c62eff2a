"""Pins of the candidate selection (Sec. 2.3.1, 3.3-3.4) and the saved
cutouts of the oracle."""

import numpy as np

from oracle.alert import cutouts, select, sigma_dm


def test_sigma_dm_is_root_of_sigma00():
    """sigma_DM = sqrt((L L^T)_00) = |L_00| for an explicit lower-triangular L
    written out by hand and packed row by row."""
    Lm = np.array([[2.5, 0, 0, 0], [0.3, 1.2, 0, 0], [-0.7, 0.1, 0.9, 0], [0.2, -0.4, 0.05, 1.7]])
    packed = np.array([[2.5, 0.3, 1.2, -0.7, 0.1, 0.9, 0.2, -0.4, 0.05, 1.7]])
    Sigma = Lm @ Lm.T
    assert abs(sigma_dm(packed)[0] - np.sqrt(Sigma[0, 0])) < 1e-15
    assert abs(sigma_dm(packed)[0] - 2.5) < 1e-15


def test_select_against_brute_force():
    rng = np.random.default_rng(3)
    n = 200
    mu = rng.uniform(0, 150, (n, 4))
    L = rng.normal(0, 1, (n, 10))
    L[:, 0] = rng.choice([5.0, 10.0, 60.0, 80.0, 20.0], n)     # ties in sigma
    L[5, 0] = np.nan
    mu[7, 0] = np.nan
    order, sg = select(mu, L, 50.0, 50.0)
    brute = []
    for i in range(n):
        if mu[i, 0] > 50.0 and abs(L[i, 0]) <= 50.0:
            brute.append((abs(L[i, 0]), i))
    brute.sort()
    assert order == [i for _, i in brute]
    assert 5 not in order and 7 not in order


def test_cutouts_edges_and_missing_steps():
    B, H, W = 2, 5, 6
    cache = {3: np.arange(B * H * W, dtype=np.float32).reshape(B, H, W)}
    out, have = cutouts(cache, {}, row=0, col=5, half=1, t_first=2, n_steps=2, B=B, H=H, W=W)
    assert list(have) == [False, True]
    assert np.all(out[0] == 0)
    # box rows -1..1, cols 4..6 of step 3: only rows 0..1, cols 4..5 inside
    exp = np.zeros((B, 3, 3), np.float32)
    exp[:, 1:3, 0:2] = cache[3][:, 0:2, 4:6]
    assert np.array_equal(out[1], exp)
