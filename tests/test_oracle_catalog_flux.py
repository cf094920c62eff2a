"""Pins of the oracle's association, monitoring and flux (Sec. 2.2)."""

import math

import numpy as np

import synth
from oracle.catalog import Catalog, dedupe, priority_order
from oracle.config import OracleConfig
from oracle.flux import box_max, measure
from oracle.pipeline import OracleStream


def pk(b, i, j, x):
    return (b, i, j, float(np.float32(x)), 0.0, 1.0, x)


def test_priority_order_ties():
    peaks = [pk(1, 5, 5, 3.0), pk(0, 9, 9, 3.0), pk(0, 2, 2, 7.0), pk(0, 9, 1, 3.0)]
    assert priority_order(peaks) == [2, 3, 1, 0]


def test_dedupe_keeps_brightest_across_bands():
    # same source in 3 bands within 2 px, a separate one 10 px away
    peaks = [pk(0, 10, 10, 5.0), pk(1, 11, 11, 9.0), pk(2, 10, 12, 6.0), pk(0, 20, 10, 4.0)]
    assert dedupe(peaks, 3.0) == [1, 3]
    # a chain: a kept peak suppresses only its own neighbours (greedy, not transitive)
    peaks = [pk(0, 0, 0, 9.0), pk(0, 0, 3, 8.0), pk(0, 0, 6, 7.0)]
    assert dedupe(peaks, 3.0) == [0, 2]


def test_association_nearest_unmatched_and_ids():
    cat = Catalog(max_sources=100, n_mon=31, r_dup=3.0, r_assoc=3.0)
    new, ended, meas, dropped = cat.step(0, [pk(0, 10, 10, 5.0), pk(0, 40, 40, 6.0)])
    assert new == [0, 1] or new == [1, 0]
    assert cat.sources[new[0]].row == 40   # brighter peak opens first -> id 0
    # next step: a peak 2 px from source (10,10) re-detects it, far peak opens id 2
    new, ended, meas, dropped = cat.step(1, [pk(3, 12, 10, 4.0), pk(0, 100, 100, 4.5)])
    assert new == [2]
    assert cat.sources[1].t_last_det == 1 and cat.sources[0].t_last_det == 0
    assert meas == [0, 1, 2]


def test_two_peaks_compete_for_one_source():
    cat = Catalog(max_sources=100, n_mon=31, r_dup=3.0, r_assoc=5.0)
    cat.step(0, [pk(0, 50, 50, 5.0)])        # id 0 at (50,50)
    # two kept peaks (4 px apart > r_dup) both within r_assoc of source 0:
    # the brighter takes it, the other opens a new source
    new, *_ = cat.step(1, [pk(0, 48, 50, 6.0), pk(0, 52, 50, 7.0)])
    assert new == [1] and cat.sources[1].row == 48
    assert cat.sources[0].t_last_det == 1


def test_episode_end_and_release():
    cat = Catalog(max_sources=100, n_mon=31, r_dup=3.0, r_assoc=3.0)
    cat.step(100, [pk(0, 5, 5, 5.0)])
    for t in range(101, 131):
        new, ended, meas, _ = cat.step(t, [])
        assert ended == [] and meas == [0]
    new, ended, meas, _ = cat.step(131, [])        # 131 - 100 == n_mon: last measured step
    assert ended == [0] and meas == [0] and cat.sources[0].t_end == 131
    new, ended, meas, _ = cat.step(132, [])
    assert ended == [] and meas == [] and 0 not in cat.sources


def test_gap_ends_episode_at_last_measured_step():
    cat = Catalog(max_sources=100, n_mon=31, r_dup=3.0, r_assoc=3.0)
    cat.step(0, [pk(0, 5, 5, 5.0)])
    new, ended, meas, _ = cat.step(50, [pk(0, 5, 5, 5.0)])
    assert ended == [0] and cat.sources[0].t_end == 31
    assert new == [1]            # the old episode is over, so a new source opens


def test_capacity_drops():
    cat = Catalog(max_sources=2, n_mon=31, r_dup=3.0, r_assoc=3.0)
    new, ended, meas, dropped = cat.step(0, [pk(0, 0, 0, 5.0), pk(0, 10, 0, 6.0), pk(0, 20, 0, 7.0)])
    assert dropped == 1 and len(new) == 2
    assert sorted(cat.sources[i].row for i in new) == [10, 20]


def test_box_max_flux_closed_form():
    """Noise-free PSF at an integer centre: flux = A; at a sub-pixel offset
    (dx, dy) the box maximum is the sample nearest the centre."""
    sp = synth.SIGMA_PSF
    A = 7.0
    for dx, dy in [(0.0, 0.0), (0.3, -0.2), (0.49, 0.49)]:
        img = np.zeros((41, 41))
        ii = np.arange(41)[:, None]
        jj = np.arange(41)[None, :]
        img = A * np.exp(-((ii - 20 - dy) ** 2 + (jj - 20 - dx) ** 2) / (2 * sp * sp))
        f = box_max(img.astype(np.float32), 20, 20, 2)
        expect = A * math.exp(-(dx * dx + dy * dy) / (2 * sp * sp))
        assert abs(f - expect) < 1e-6 * A
    # box clipped by the image edge
    img = np.zeros((5, 5), dtype=np.float32)
    img[0, 0] = 3.0
    assert box_max(img, 1, 1, 2) == 3.0 and box_max(img, 4, 4, 2) == 0.0
    assert list(measure(np.stack([img, 2 * img]), 0, 0, 1)) == [3.0, 6.0]


def test_backfill_and_window_of_single_detection():
    """A source seen once at t_d is measured on [t_d - 32, t_d + 31]: its
    64-step window is exactly the backfill, the detection and the monitoring,
    each cell the 5x5 box maximum of that step's image."""
    B, H, W = 2, 64, 64
    cfg = OracleConfig(B=B, H=H, W=W, s=3.0, kappa=7.0, t_bf=32, n_mon=31)
    orc = OracleStream(cfg)
    rng = np.random.default_rng(0)
    t_d = 40
    frames = {}
    for t in range(0, t_d + 32):
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        if t == t_d:
            cube[0, 30, 30] += 20.0   # bright, yet below the pixel QC threshold
        frames[t] = cube
        orc.ingest(t, cube)
        orc.detect()
        orc.extract_flux()
        if t == t_d:
            assert orc.last["new"] == [0]
        else:
            assert orc.last["new"] == []
    assert orc.last["ended"] == [0] and orc.catalog.sources[0].t_end == t_d + 31
    grid, valid = orc.spectrum(0)
    assert valid.all()
    for c, tau in enumerate(range(t_d - 32, t_d + 32)):
        for b, row in ((0, 0), (1, 8)):       # band 1 of 2 sits on grid row 8
            assert grid[row, c] == frames[tau][b, 28:33, 28:33].max()
    assert not grid[[r for r in range(16) if r not in (0, 8)]].any()
