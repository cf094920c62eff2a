"""Pins of the oracle's quality control (App. A)."""

import numpy as np
import pytest

import synth
from oracle.config import OracleConfig
from oracle.pipeline import OracleStream
from oracle.qc import RunningStats, band_reject, band_stats, robust_z


def test_band_stats_closed_form():
    cube = np.zeros((3, 4, 5), dtype=np.float32)
    cube[0] = 2.0
    cube[1, 0, 0] = 20.0
    cube[2] = np.arange(20, dtype=np.float32).reshape(4, 5)
    mean, rms, nf = band_stats(cube)
    assert mean[0] == 2.0 and rms[0] == 2.0
    assert mean[1] == 1.0 and abs(rms[1] - np.sqrt(400.0 / 20)) < 1e-15
    assert mean[2] == 9.5 and abs(rms[2] ** 2 - sum(v * v for v in range(20)) / 20) < 1e-12
    assert list(nf) == [0, 0, 0]


@pytest.mark.parametrize("B,seed", [(4, 0), (7, 1), (16, 2)])
def test_robust_z_vs_numpy_median(B, seed):
    v = np.random.default_rng(seed).standard_normal(B)
    z = robust_z(v, np.ones(B, dtype=bool))
    med = np.median(v)
    mad = np.median(np.abs(v - med))
    assert np.allclose(z, (v - med) / mad, rtol=0, atol=1e-15)


def test_robust_z_hand_cases():
    # even count: median of (1,2,3,10) is 2.5; |d| = 1.5,0.5,0.5,7.5 -> MAD 1.0
    z = robust_z(np.array([1.0, 2.0, 3.0, 10.0]), np.ones(4, dtype=bool))
    assert np.allclose(z, [-1.5, -0.5, 0.5, 7.5])
    # MAD = 0: equal-to-median bands score 0, others +inf
    z = robust_z(np.array([5.0, 5.0, 5.0, 6.0, 5.0]), np.ones(5, dtype=bool))
    assert list(z[:3]) == [0.0, 0.0, 0.0] and z[3] == np.inf and z[4] == 0.0


def test_nonfinite_band_rejected_and_excluded():
    rng = np.random.default_rng(0)
    cube = rng.standard_normal((6, 32, 32)).astype(np.float32)
    cube[2, 5, 5] = np.nan
    cube[4, 0, 1] = np.inf
    rej, *_ = band_reject(cube, 5.0, 5.0)
    assert rej == (1 << 2) | (1 << 4)


def test_welford_vs_two_pass():
    rng = np.random.default_rng(1)
    frames = rng.standard_normal((23, 2, 6, 7)) * 3.0 + 1.5
    st = RunningStats(2, 6, 7)
    for f in frames:
        for b in range(2):
            st.update(b, f[b])
    assert np.allclose(st.mean, frames.mean(axis=0), atol=1e-13)
    var = frames.var(axis=0, ddof=1)
    assert np.allclose(st.m2 / (st.n[:, None, None] - 1), var, rtol=1e-12, atol=1e-13)


def test_rms_floor():
    # RMS values 1.000, 1.001, ..., one band at 1.02: MAD ~ 0.0005 would give
    # z ~ 40; the 5 % floor of the median scale gives z = 0.02 / 0.05 < 5.
    v = np.array([1.0, 1.001, 0.999, 1.0005, 0.9995, 1.02])
    z = robust_z(v, np.ones(6, dtype=bool), 0.05)
    med = np.median(v)
    assert abs(z[5] - (1.02 - med) / (0.05 * med)) < 1e-12 and abs(z[5]) < 5
    z = robust_z(np.array([1.0, 1.0, 1.0, 5.0]), np.ones(4, dtype=bool), 0.05)
    assert abs(z[3] - 80.0) < 1e-12


def test_pixel_zeta_hand_case():
    st = RunningStats(1, 1, 2)
    for v in (1.0, 3.0, 1.0, 3.0):   # mean 2, sample sd sqrt(4/3)
        st.update(0, np.array([[v, v]]))
    M = np.ones((1, 2), dtype=bool)
    z = st.zeta_max(0, np.array([[2.0, 6.0]]), M, 4)
    assert abs(z - 4.0 / np.sqrt(4.0 / 3.0)) < 1e-12
    assert st.zeta_max(0, np.array([[2.0, 6.0]]), M, 5) == 0.0   # not yet armed


@pytest.mark.slow
def test_rfi_recall_and_clean_false_rejections():
    """Every injected RFI (step, band) is discarded; clean bands rarely are."""
    spec = synth.spec_streaming(T=40, H=1024)
    spec.rfi_p = 0.08
    spec.n_sources = 40
    st = synth.Stream(spec)
    cfg = OracleConfig(B=spec.B, H=spec.H, W=spec.W, sky_mask=st.mask, freqs_mhz=st.freqs)
    orc = OracleStream(cfg)
    false_rej = clean = 0
    n_rfi = 0
    for t in range(spec.T):
        rej = orc.ingest(t, st.frame(t))
        truth = st.rfi_mask(t)
        n_rfi += bin(truth).count("1")
        assert rej & truth == truth, (t, bin(rej), bin(truth))
        false_rej += bin(rej & ~truth).count("1")
        clean += spec.B - bin(truth).count("1")
    assert n_rfi > 20
    assert false_rej <= 0.01 * clean
