"""Detection variants through the C ABI against the FP64 oracle: the circular
uniform kernel (Sec. 2.1.1), the PSF pre-filter (the matched filter of a point
source, detection on the PSF-correlated image) and the background-subtracted
flux (box maximum minus the mean of the surrounding annulus)."""

import numpy as np
import pytest

import synth
from oracle.filters import centre_spread, correlate_2d
from oracle.detect import band_peaks

from parity import compare_events, dev_peaks_as_oracle, make_pair, run_steps

pytestmark = pytest.mark.gpu


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _frames(rng, B, H, W, mask, n, n_src=6):
    ii, jj = np.mgrid[0:H, 0:W]
    out = []
    for _ in range(n):
        cube = rng.standard_normal((B, H, W)) + 0.2
        for _ in range(n_src):
            b = int(rng.integers(B))
            ci, cj = rng.uniform(10, H - 10), rng.uniform(10, W - 10)
            cube[b] += rng.uniform(6.0, 25.0) * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2 * 1.274 ** 2))
        cube = cube.astype(np.float32)
        if mask is not None:
            cube *= mask
        out.append(cube)
    return out


@pytest.mark.parametrize("k,W,masked", [(3, 201, True), (8, 196, True), (24, 150, False), (24, 260, True)])
def test_disk_kernel_planes_peaks_events(k, W, masked):
    """Dense C and S planes (scale-aware 1e-5), peaks (bracketing at kappa
    +- 1e-3), events and spectra over three steps on ragged images (H not a
    multiple of the 32-row tile, W not a multiple of 64), with and without a
    sky mask."""
    _torch_cuda()
    rng = np.random.default_rng(100 + k + W)
    B, H = 3, 150
    mask = synth.sky_mask(H, W) if masked else None
    ctx, orc = make_pair(B, H, W, sky_mask=mask, debug_planes=1, kernel=2, bg_halfwidth=k, kappa=4.0,
                         monitor_steps=2, backfill_steps=2)
    res = run_steps(ctx, orc, _frames(rng, B, H, W, mask, 3), [0, 1, 2], compare_planes=True,
                    label=f"disk-k{k}-W{W}")
    # (at radius 3 a blob dominates its own 29-pixel disk, so few pixels pass)
    assert res["steps"] == 3 and (k < 8 or res["events"] > 0), res


def test_disk_kernel_tiny_workload():
    """The tiny workload (4 x 256^2, 16 steps) with the disk of radius 24."""
    _torch_cuda()
    st = synth.Stream(synth.spec_tiny())
    s = st.spec
    ctx, orc = make_pair(s.B, s.H, s.W, kernel=2)
    res = run_steps(ctx, orc, [st.frame(t) for t in range(s.T)], list(range(s.T)), label="disk-tiny")
    assert res["steps"] == s.T and res["spectra"] > 0, res


def test_background_subtracted_flux_bitwise():
    """Flux = box maximum minus the float64 mean of the annulus 3 px wide
    around the 5 x 5 box, rounded once: dynamic spectra bitwise equal to the
    oracle's on the tiny workload (sources near the image edge included by
    the generator's placement box)."""
    _torch_cuda()
    st = synth.Stream(synth.spec_tiny())
    s = st.spec
    ctx, orc = make_pair(s.B, s.H, s.W, flux_bg_width=3)
    res = run_steps(ctx, orc, [st.frame(t) for t in range(s.T)], list(range(s.T)), label="bgflux")
    assert res["steps"] == s.T and res["spectra"] > 0, res


def _psf_scale(X, M, g):
    w = M.astype(np.float64)
    den = correlate_2d(w, g)
    return np.where(den > 0, correlate_2d(w * np.abs(X.astype(np.float64)), g) / np.where(den > 0, den, 1.0), 0.0)


@pytest.mark.parametrize("masked", [True, False])
def test_psf_prefilter_detection(masked):
    """Detection on the PSF-correlated image D = (G_psf * (M X)) / (G_psf * M)
    (PSF width 1.274 px, half-width 6): the device's D at 1e-5 of its scale
    (G_psf * (M |X|)) / (G_psf * M); every listed peak a local maximum of the
    oracle's D up to twice that tolerance and above kappa - 1e-3 in the
    oracle's statistics of D; every oracle peak with margins beyond those
    tolerances listed; events exact with the oracle's catalogue fed the
    device's validated list; spectra (flux on the unfiltered image) bitwise."""
    _torch_cuda()
    rng = np.random.default_rng(5 if masked else 6)
    B, H, W = 3, 160, 200
    mask = synth.sky_mask(H, W) if masked else None
    kappa, delta = 4.0, 1e-3
    ctx, orc = make_pair(B, H, W, sky_mask=mask, psf_sigma=1.274, kappa=kappa, monitor_steps=2, backfill_steps=2)
    M = orc.M
    c = orc.cfg
    n_peaks = n_spec = 0
    for t, cube in enumerate(_frames(rng, B, H, W, mask, 4, n_src=10)):
        print(f"psf masked={masked} step t={t}", flush=True)
        rej = orc.ingest(t, cube)
        assert ctx.ingest(t, cube, want_rejected=True) == rej
        pd, ev, _ = ctx.detect()
        Dd = ctx.debug_read("prefiltered")
        Do64 = np.stack([centre_spread(orc.cache[t][b], M, orc.g_psf)[0] for b in range(B)])
        Do = Do64.astype(np.float32)
        listed = {}
        for b in range(B):
            if rej >> b & 1:
                continue
            sc = _psf_scale(orc.cache[t][b], M, orc.g_psf)
            err = np.abs(Dd[b].astype(np.float64) - Do64[b])
            assert np.all(err[M] <= 1e-5 * sc[M] + 1e-30), (t, b, float((err / np.maximum(sc, 1e-30))[M].max()))
            tol = 2e-5 * sc + 1e-30
            # oracle statistics of its own D at kappa -+ delta
            lo = {(p[1], p[2]) for p in band_peaks(b, Do[b], M, orc.g, kappa - delta, 1, c.k_peak)[0]}
            hi = {(p[1], p[2]) for p in band_peaks(b, Do[b], M, orc.g, kappa + delta, 1, c.k_peak)[0]}
            C, S, _ = centre_spread(Do[b], M, orc.g)
            got = {(int(p["row"]), int(p["col"])) for p in pd if int(p["band"]) == b}
            listed[b] = got
            for (i, j) in got:
                r0, r1 = max(0, i - 3), min(H, i + 4)
                c0, c1 = max(0, j - 3), min(W, j + 4)
                win = np.where(M[r0:r1, c0:c1], Do64[b, r0:r1, c0:c1], -np.inf)
                assert M[i, j] and Do64[b, i, j] >= win.max() - 2 * tol[i, j], (t, b, i, j, "not a local maximum")
                sig = (Do64[b, i, j] - C[i, j]) / np.sqrt(S[i, j]) if S[i, j] > 0 else np.inf
                assert sig > kappa - delta - 1e-4, (t, b, i, j, sig)
            for (i, j) in hi - got:
                r0, r1 = max(0, i - 3), min(H, i + 4)
                c0, c1 = max(0, j - 3), min(W, j + 4)
                win = np.where(M[r0:r1, c0:c1], Do64[b, r0:r1, c0:c1], -np.inf)
                win[i - r0, j - c0] = -np.inf
                assert Do64[b, i, j] - win.max() <= 2 * tol[i, j], (t, b, i, j, "missing peak")
            assert lo >= hi
            n_peaks += len(got)
        # association from the device's validated list; flux reads the unfiltered cache
        _, new_o, ended_o = orc.associate(dev_peaks_as_oracle(pd), 0)
        compare_events(ev, orc, new_o, ended_o, f"psf t={t}")
        orc.extract_flux()
        ctx.extract_flux()
        rows = [c.grid_row(b) for b in range(B)]
        for sid in list(orc.catalog.sources):
            grid, valid = orc.spectrum(sid)
            out, vd, _ = ctx.read_spectrum(sid)
            assert np.array_equal(vd, valid) and np.array_equal(out, np.where(valid, grid[rows], 0.0).astype(np.float32))
            n_spec += 1
    print(f"psf masked={masked}: peaks {n_peaks}, spectra {n_spec}", flush=True)
    assert n_peaks > 10 and n_spec > 0
