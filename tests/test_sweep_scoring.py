"""Host-side scoring of the accuracy sweep (Sec. 3.1 definitions of P, R,
F1 and F90) on hand-made cases."""

import numpy as np

from paper_2103_15418_amd.sweep import accumulate, match, scores


def test_match_greedy_by_flux_nearest_peak():
    # two sources 4 px apart, one peak between them (2 px from each) and one far peak:
    # the brighter source takes the shared peak, the fainter one is missed
    peaks_r, peaks_c = [10, 50], [12, 50]
    got, taken = match(peaks_r, peaks_c, [10, 10], [10, 14], [5.0, 9.0], r_match=3.0)
    assert list(got) == [-1, 0] and list(taken) == [True, False]


def test_scores_per_bin_and_f90():
    edges = (0.0, 1.0, 2.0, np.inf)
    counts = {}
    # bin 0: 4 true, 1 found; bin 1: 2 true, 2 found; bin 2: 3 true, 3 found
    got = np.array([0, -1, -1, -1, 1, 2, 3, 4, 5])
    snr = np.array([0.5, 0.2, 0.7, 0.9, 1.5, 1.2, 5.0, 7.0, 9.0])
    taken = np.array([True] * 6 + [False, False])
    sig = np.array([0.5, 1.5, 1.2, 5.0, 7.0, 9.0, 0.3, 1.7])   # two false positives in bins 0, 1
    accumulate(counts, got, taken, snr, sig, edges)
    s = scores(counts, edges)
    assert s["recall"] == [0.25, 1.0, 1.0]
    assert s["precision"] == [0.5, 2 / 3, 1.0]
    f1 = [2 * 0.5 * 0.25 / 0.75, 2 * (2 / 3) / (5 / 3), 1.0]
    assert np.allclose(s["f1"], f1)
    assert s["F90"] == 2.0
