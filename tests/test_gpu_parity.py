"""Device path (through the C ABI) against the FP64 oracle on seeded synthetic
streams.  Tolerances are documented in tests/parity.py."""

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
from oracle.filters import taps_1d

from parity import check_centre_sampled, check_welford, cnn_scale, make_pair, run_steps

pytestmark = pytest.mark.gpu


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _log(msg):
    print(msg, flush=True)


def test_planes_and_peaks_ragged_tiles_with_mask():
    """C, S dense planes and the peak list on images spanning several 64x64
    tiles with ragged tails, a circular sky mask and injected bright pixels."""
    _torch_cuda()
    rng = np.random.default_rng(0)
    B, H, W = 3, 150, 201
    mask = synth.sky_mask(H, W)
    ctx, orc = make_pair(B, H, W, sky_mask=mask, debug_planes=1, kappa=3.0, bg_sigma=4.0)
    frames, ts = [], []
    for t in range(3):
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        for _ in range(6):
            cube[rng.integers(B), rng.integers(20, H - 20), rng.integers(20, W - 20)] += 9.0
        cube *= mask
        frames.append(cube)
        ts.append(t)
    st = run_steps(ctx, orc, frames, ts, compare_planes=True, label="ragged")
    assert st["steps"] == 3


@pytest.mark.parametrize("kernel,s,k", [(0, 8.0, 0), (0, 3.0, 0), (1, 0.0, 5), (0, 5.0, 15), (0, 12.0, 36)])
def test_planes_kernel_variants(kernel, s, k):
    """Gaussian at the specialised half-widths 24/15/36, the generic path
    (k = 9) and the square box kernel."""
    _torch_cuda()
    rng = np.random.default_rng(1)
    B, H, W = 2, 130, 97
    params = dict(debug_planes=1, kernel=kernel, bg_sigma=s if s > 0 else 1.0, bg_halfwidth=k)
    ctx, orc = make_pair(B, H, W, **params)
    cube = (rng.standard_normal((B, H, W)) * 2.0 + 0.5).astype(np.float32)
    cube[0, 60, 40] += 15.0
    run_steps(ctx, orc, [cube], [0], compare_planes=True, label=f"k{kernel}-{s}-{k}")


@pytest.mark.parametrize("k,strip_h", [(24, None), (15, None), (36, None), (24, "64"), (15, "96")])
def test_strip_filters_ragged(k, strip_h, monkeypatch):
    """Float32 strip kernels (W % 4 == 0, k in {15, 24, 36}): dense C / S planes
    and peaks on a ragged image (W not a multiple of 64, H not a multiple of
    32) with a sky mask, at the default strip height and at forced heights
    that give several 32-row chunks per strip."""
    _torch_cuda()
    if strip_h is not None:
        monkeypatch.setenv("LPF_STRIP_H", strip_h)
    rng = np.random.default_rng(7 + k)
    B, H, W = 3, 150, 196
    mask = synth.sky_mask(H, W)
    ctx, orc = make_pair(B, H, W, sky_mask=mask, debug_planes=1, kappa=3.5, bg_halfwidth=k,
                         bg_sigma=k / 3.0)
    frames = []
    for t in range(2):
        cube = (rng.standard_normal((B, H, W)) + 0.3).astype(np.float32)
        for _ in range(5):
            cube[rng.integers(B), rng.integers(10, H - 10), rng.integers(10, W - 10)] += 10.0
        frames.append(cube * mask)
    run_steps(ctx, orc, frames, [0, 1], compare_planes=True, label=f"strip-k{k}-h{strip_h}")


def _clip_frames(rng, B, H, W, mask, n, n_src=14):
    """Noise with Gaussian blobs (sigma 1.5 px) of 6-30: iteration 1 clips the
    cores, later iterations the wings that the cores' spread had hidden."""
    frames = []
    ii, jj = np.mgrid[0:H, 0:W]
    for _ in range(n):
        cube = rng.standard_normal((B, H, W))
        for _ in range(n_src):
            b = int(rng.integers(B))
            ci, cj = rng.uniform(8, H - 8), rng.uniform(8, W - 8)
            cube[b] += rng.uniform(6.0, 30.0) * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2 * 1.5 ** 2))
        cube = cube.astype(np.float32)
        if mask is not None:
            cube *= mask
        frames.append(cube)
    return frames


@pytest.mark.parametrize("W,k,iters,masked,seed", [(196, 15, 2, True, 1), (201, 9, 3, True, 2),
                                                   (196, 24, 5, True, 0), (201, 24, 3, False, 0),
                                                   (200, 36, 2, True, 0)])
def test_clip_iterations(W, k, iters, masked, seed):
    """Several sigma-clip iterations (Sec. 2.1.1 repeat, App. C; clipped
    pixels leave the next iteration's statistics): the clip mask Y, C and S of
    the last iteration and the peak list P = Q and Y against the oracle's
    iterations on ragged images with and without a sky mask, the first pass
    on the strip kernels where W % 4 = 0 and later passes on the tile
    kernels; events and spectra as every other stream test.  Differences are
    allowed only in the zones around pixels whose margin lies within 1e-3 of
    the threshold in some iteration (none for these seeds, so everything is
    compared).  At five iterations one band stops before the others."""
    _torch_cuda()
    rng = np.random.default_rng(1000 * seed + W + k + iters)
    B, H = 3, 150
    mask = synth.sky_mask(H, W) if masked else None
    ctx, orc = make_pair(B, H, W, sky_mask=mask, debug_planes=1, kappa=4.0, bg_halfwidth=k,
                         bg_sigma=max(k / 3.0, 5.0), clip_iters=iters)
    frames = _clip_frames(rng, B, H, W, mask, 3)
    res = run_steps(ctx, orc, frames, [0, 1, 2], label=f"clip-W{W}-k{k}-n{iters}")
    assert res["steps"] == 3 and res["fragile"] == 0 and res["excused"] == 0, res


def test_clip_iterations_tiny_workload():
    """The tiny workload (4 x 256^2, 16 steps) with three clip iterations at
    kappa = 4.5: every step compared as in test_tiny_stream_full_pipeline."""
    _torch_cuda()
    st = synth.Stream(synth.spec_tiny())
    s = st.spec
    ctx, orc = make_pair(s.B, s.H, s.W, debug_planes=1, clip_iters=3)
    frames = [st.frame(t) for t in range(s.T)]
    res = run_steps(ctx, orc, frames, list(range(s.T)), label="tiny-clip3")
    assert res["steps"] == s.T and res["spectra"] > 0, res


def test_tiny_stream_full_pipeline():
    """4 subbands x 16 steps of 256^2 (the tiny workload): QC, peaks, events,
    dynamic spectra every step, then the network on the ended episodes."""
    torch = _torch_cuda()
    st = synth.Stream(synth.spec_tiny())
    s = st.spec
    ctx, orc = make_pair(s.B, s.H, s.W, debug_planes=1)
    frames = [st.frame(t) for t in range(s.T)]
    res = run_steps(ctx, orc, frames, list(range(s.T)), compare_planes=True, label="tiny")
    assert res["steps"] == s.T and res["resyncs"] == 0
    assert res["spectra"] > 0


def test_instrument_scale_sampled_and_lists():
    """16 x 1024^2 in the circular mask (instrument workload), first steps
    with the dense oracle: QC statistics and scores, Welford state, peak
    bracketing, events, spectra; C at sampled pixels."""
    _torch_cuda()
    spec = synth.spec_instrument(T=4)
    st = synth.Stream(spec)
    ctx, orc = make_pair(spec.B, spec.H, spec.W, sky_mask=st.mask)
    frames = [st.frame(t) for t in range(spec.T)]
    res = run_steps(ctx, orc, frames, list(range(spec.T)), label="instrument")
    assert res["steps"] == spec.T and res["resyncs"] <= 1
    check_welford(ctx, orc, "instrument")
    X = orc.cache[spec.T - 1]
    check_centre_sampled(ctx.debug_read("centre"), X, orc.M, orc.g, orc.cfg.k_bg, orc.rejected[spec.T - 1],
                         np.random.default_rng(7), n=48, label="instrument")


def _qc_stream(T=16, H=256):
    spec = synth.spec_streaming(T=T, H=H)
    spec.n_sources = 10
    spec.rfi_p = 0.1
    spec.rfi_from_t = 2
    return synth.Stream(spec)


def test_qc_rejects_rfi_and_nonfinite_like_oracle():
    """Streaming-style RFI (stripes, x5 noise) from step 2, a NaN pixel at
    step 5 and, after the pixel test has armed (8 accepted steps), a single
    +40 pixel in a clean band at step 12 that only the running z catches:
    the same decisions as the oracle, band mean / RMS at 1e-12, their robust
    z at 1e-9 and max |zeta| at 1e-5 every step, rejected bands without
    peaks, Welford state of the accepted steps."""
    _torch_cuda()
    st = _qc_stream()
    spec = st.spec
    ctx, orc = make_pair(spec.B, spec.H, spec.W, sky_mask=st.mask, qc_warmup=8)
    frames = [st.frame(t) for t in range(spec.T)]
    frames[5][3, 100, 100] = np.nan
    zeta_band = next(b for b in range(spec.B) if (12, b) not in st.rfi)
    frames[12][zeta_band, 128, 130] += 40.0
    res = run_steps(ctx, orc, frames, list(range(spec.T)), label="rfi")
    assert res["steps"] == spec.T, res
    assert res["zeta_checked"] >= 8 * spec.B // 2, res
    # every injected RFI band-step rejected; the +40 pixel rejected by zeta alone
    for t in range(spec.T):
        assert orc.rejected[t] & st.rfi_mask(t) == st.rfi_mask(t), t
    check_welford(ctx, orc, "rfi")


def test_qc_zeta_alone_rejects():
    """The pixel test by itself: after warm-up a clean band gains one +40
    pixel; its band mean and RMS z stay below 5 and its max |zeta| exceeds
    30, on both sides."""
    _torch_cuda()
    rng = np.random.default_rng(17)
    B, H, W = 6, 128, 128
    ctx, orc = make_pair(B, H, W, qc_warmup=8)
    frames = [rng.standard_normal((B, H, W)).astype(np.float32) for _ in range(11)]
    frames[10][2, 64, 70] += 40.0
    run_steps(ctx, orc, frames, list(range(11)), label="zeta")
    L = orc.last
    assert orc.rejected[10] == 1 << 2
    assert abs(L["z_mean"][2]) < 5 and abs(L["z_rms"][2]) < 5 and L["zeta"][2] > 30
    assert ctx.debug_read("bandstats")[2, 4] > 30


def test_gap_in_time_and_backfill():
    """Steps with a gap: missing steps stay invalid in the spectra."""
    _torch_cuda()
    rng = np.random.default_rng(3)
    B, H, W = 2, 96, 96
    ctx, orc = make_pair(B, H, W, kappa=6.0, bg_sigma=3.0, backfill_steps=8, monitor_steps=5)
    ts = [0, 1, 2, 5, 6, 7, 9, 10, 11, 12, 20, 21]
    frames = []
    for t in ts:
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        if t in (7, 21):
            cube[1, 40, 50] += 25.0
        frames.append(cube)
    res = run_steps(ctx, orc, frames, ts, label="gap")
    assert res["steps"] == len(ts) and res["events"] >= 2


@pytest.mark.parametrize("W", [72, 70])
def test_flux_boxes_at_image_edges(W):
    """Sources on the first and last rows and columns: the flux boxes are
    clipped to the image (W = 72: two aligned 16-byte loads per box row,
    clamped at 0 and W - 8; W = 70: the scalar path); fluxes, backward fills
    and spectra bitwise equal to the oracle's."""
    _torch_cuda()
    rng = np.random.default_rng(11)
    B, H = 2, 64
    # a wide background kernel, so that a corner source's own share of the
    # clipped spread leaves it above kappa (the oracle finds all seven; the
    # last two merge within dup_radius): six open at t = 4 with four steps of
    # backward fill, are measured at 5 .. 7 and end at 8
    ctx, orc = make_pair(B, H, W, kappa=6.0, bg_sigma=8.0, backfill_steps=4, monitor_steps=3)
    spots = [(0, 0), (1, W - 1), (H - 1, 2), (30, 1), (33, W - 2), (H - 2, W - 3), (H - 1, W - 1)]
    frames, ts = [], list(range(9))
    for t in ts:
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        if t in (4, 5):
            for q, (r, c) in enumerate(spots):
                cube[q % B, r, c] += 30.0 + 2.0 * q
        frames.append(cube)
    res = run_steps(ctx, orc, frames, ts, label=f"edges W={W}")
    assert res["steps"] == len(ts) and res["events"] >= 12 and res["resyncs"] == 0


def test_association_conflicts_and_duplicates():
    """Catalogue cases that take the sequential resolutions: two kept peaks
    (farther apart than dup_radius) both within assoc_radius of one live
    source, a duplicate pair across bands, and a peak with two sources in
    reach; events and lists must match the oracle at every step."""
    _torch_cuda()
    rng = np.random.default_rng(21)
    B, H, W = 2, 96, 96
    ctx, orc = make_pair(B, H, W, kappa=6.0, bg_sigma=3.0, backfill_steps=4, monitor_steps=3)
    frames, ts = [], list(range(6))
    for t in ts:
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        if t == 0:
            cube[0, 50, 50] += 30.0            # source A
            cube[1, 20, 20] += 30.0            # source B
            cube[0, 20, 25] += 28.0            # source C (5 px from B)
        if t == 1:
            cube[0, 50, 47] += 35.0            # both 3 px from A, 6 px apart:
            cube[1, 50, 53] += 32.0            #   the brighter takes A, the other opens
            cube[0, 20, 22] += 33.0            # within reach of B (2 px) and C (3 px)
            cube[1, 21, 22] += 31.0            # duplicate of the previous one (1.4 px)
        frames.append(cube)
    res = run_steps(ctx, orc, frames, ts, label="conflicts")
    assert res["steps"] == len(ts) and res["events"] >= 5 and res["resyncs"] == 0


@pytest.mark.parametrize("n,maxb", [(37, 64), (100, 128)])
def test_network_fp32_parity_ragged_batch(n, maxb):
    """infer_windows on 37 and 100 seeded windows (ragged multiples of 32;
    up to 64 windows fc1 splits the outputs over two workgroups per K chunk,
    above it runs a workgroup per 32 windows) against the FP64 oracle
    network, per output within 1e-5 of the condition scale."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Model
    wts = synth.cnn_weights(seed=11, leaky_alpha=0.1)
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((n, 16, 64)) * 2.0).astype(np.float32)
    x[::3, 5, 20:30] += 6.0
    m = Model(wts, max_batch=maxb)
    mu_d, L_d = m.infer_windows(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    raw = ocnn.forward_raw(x.astype(np.float64), wts)
    mu_o, L_o = ocnn.head(raw)
    sc = cnn_scale(x.astype(np.float64), wts)
    assert np.all(np.abs(mu_d.cpu().numpy() - mu_o) <= 1e-5 * sc[:, :4] + 1e-6)
    assert np.all(np.abs(L_d.cpu().numpy() - L_o) <= 1e-5 * sc[:, 4:] + 1e-6)


def test_network_on_ended_episodes_matches_oracle():
    """lpf_infer over the episodes that ended at a step: same ids and outputs
    as the oracle network applied to the oracle's windows."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Model
    rng = np.random.default_rng(5)
    B, H, W = 4, 80, 80
    ctx, orc = make_pair(B, H, W, kappa=6.0, bg_sigma=3.0, backfill_steps=6, monitor_steps=4)
    wts = synth.cnn_weights(seed=2)
    model = Model(wts, max_batch=8)
    checked = 0
    for t in range(14):
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        if t in (3, 4):
            cube[:, 30, 30] += 20.0
            cube[:, 60, 15] += 18.0
        orc.ingest(t, cube)
        ctx.ingest(t, cube)
        orc.detect()
        ctx.detect()
        orc.extract_flux()
        ctx.extract_flux()
        mu_o, L_o, ids_o = orc.infer(wts)
        mu_d, L_d, src = model.infer([ctx])
        assert [int(s[1]) for s in src] == list(ids_o), t
        if ids_o:
            x = np.stack([orc.spectrum(s)[0] for s in ids_o])
            sc = cnn_scale(x, wts)
            assert np.all(np.abs(mu_d - mu_o) <= 1e-5 * sc[:, :4] + 1e-6)
            assert np.all(np.abs(L_d - L_o) <= 1e-5 * sc[:, 4:] + 1e-6)
            checked += len(ids_o)
    assert checked >= 2


def test_async_inference_lagged_and_batch_overflow():
    """lpf_infer_async / lpf_infer_collect: results collected one step late
    equal the oracle's for that step; more ended episodes than the model's
    batch are reported by collect (EFULL) while lpf_infer falls back to
    host-driven chunks and returns them all; at most four tickets."""
    _torch_cuda()
    from paper_2103_15418_amd import LpfError, Model
    rng = np.random.default_rng(11)
    B, H, W = 4, 96, 96
    ctx, orc = make_pair(B, H, W, kappa=6.0, bg_sigma=3.0, backfill_steps=6, monitor_steps=4)
    wts = synth.cnn_weights(seed=4)
    big = Model(wts, max_batch=16)
    small = Model(wts, max_batch=8)
    spots = [(12 + 24 * i, 12 + 24 * j) for i in range(4) for j in range(4)][:12]
    pending = None
    checked = overflow_steps = 0

    def compare(res, ref, label):
        mu_d, L_d, src = res
        mu_o, L_o, ids_o, x = ref
        assert [int(s[1]) for s in src] == list(ids_o), label
        if ids_o:
            sc = cnn_scale(x, wts)
            assert np.all(np.abs(mu_d - mu_o) <= 1e-5 * sc[:, :4] + 1e-6), label
            assert np.all(np.abs(L_d - L_o) <= 1e-5 * sc[:, 4:] + 1e-6), label

    for t in range(12):
        cube = rng.standard_normal((B, H, W)).astype(np.float32)
        if t == 3:
            for (r, c) in spots:
                cube[:, r, c] += 25.0
        orc.ingest(t, cube)
        ctx.ingest(t, cube)
        orc.detect()
        ctx.detect()
        orc.extract_flux()
        ctx.extract_flux()
        mu_o, L_o, ids_o = orc.infer(wts)
        x = np.stack([orc.spectrum(s)[0] for s in ids_o]) if ids_o else None
        ref = (mu_o, L_o, ids_o, x)
        tk = big.infer_async([ctx])                    # collected at the next step
        if len(ids_o) > small.max_batch:
            overflow_steps += 1
            t_small = small.infer_async([ctx])
            with pytest.raises(LpfError) as err:
                small.collect(t_small)
            assert err.value.code == -3                # LPF_EFULL
            compare(small.infer([ctx]), ref, f"fallback t={t}")
        if pending is not None:
            compare(big.collect(pending[0]), pending[1], f"lagged t={t - 1}")
            checked += len(pending[1][2])
        pending = (tk, ref)
    compare(big.collect(pending[0]), pending[1], "last")
    checked += len(pending[1][2])
    assert checked >= 12 and overflow_steps >= 1
    # ticket limit: four outstanding, the fifth is refused
    tks = [big.infer_async([ctx]) for _ in range(4)]
    with pytest.raises(LpfError) as err:
        big.infer_async([ctx])
    assert err.value.code == -3
    for tk in reversed(tks):                           # any collection order
        big.collect(tk)
    with pytest.raises(LpfError):
        big.collect(tks[0])                            # already collected
