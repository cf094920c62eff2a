"""Full-size workloads in the configuration the benchmark times (pipelined
ingest, no debug planes), compared through the C ABI with the FP64 oracle on
outputs it can compute one by one: QC statistics and decisions every step,
the validity of every listed peak and completeness on random tiles, C at
sampled pixels, then events (exact) and dynamic spectra (bitwise) with the
oracle's catalogue fed the validated peak list, the Welford state and the
network on the episodes that end."""

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn

from parity import check_welford, cnn_scale, make_pair, run_steps_sampled

pytestmark = pytest.mark.gpu


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_instrument_workload_40_steps_with_network():
    """16 x 1024^2 in the circular mask, 50 dispersed sources, steps 0-39:
    the pixel test arms (8 accepted steps), episodes end (t_last_det + 31)
    and their windows go through the FP32 network, compared with the oracle
    network on the oracle's windows (1e-5 of the condition scale)."""
    _torch_cuda()
    from paper_2103_15418_amd import Model
    spec = synth.spec_instrument(T=40)
    st = synth.Stream(spec)
    ctx, orc = make_pair(spec.B, spec.H, spec.W, sky_mask=st.mask, pipeline_ingest=1)
    wts = synth.cnn_weights()
    model = Model(wts, max_batch=256)
    inferred = [0]

    def on_step(t, stats):
        mu_o, L_o, ids_o = orc.infer(wts)
        mu_d, L_d, src = model.infer([ctx])
        assert [int(s[1]) for s in src] == list(ids_o), t
        if ids_o:
            x = np.stack([orc.spectrum(s)[0] for s in ids_o])
            sc = cnn_scale(x, wts)
            assert np.all(np.abs(mu_d - mu_o) <= 1e-5 * sc[:, :4] + 1e-6), t
            assert np.all(np.abs(L_d - L_o) <= 1e-5 * sc[:, 4:] + 1e-6), t
            inferred[0] += len(ids_o)

    res = run_steps_sampled(ctx, orc, st.frame, list(range(spec.T)), label="instrument40",
                            check_welford_at=(spec.T - 1,), on_step=on_step)
    assert res["steps"] == spec.T and res["zeta_checked"] > 0 and res["ended"] > 0, res
    assert inferred[0] == res["ended"] and res["spectra"] > 500, (inferred, res)


def test_streaming_workload_2048_with_rfi():
    """16 x 2048^2 in the circular mask (streaming workload) for 12 steps,
    RFI on 10 % of (band, step) from step 4 (the workload's rate is 5 % from
    step 8; raised so that RFI falls inside the run), 200 sources: every RFI
    band rejected, the pixel test armed from step 8, peaks, events, spectra
    and the Welford state at full size."""
    _torch_cuda()
    spec = synth.spec_streaming(T=12)
    spec.rfi_p = 0.10
    spec.rfi_from_t = 4
    st = synth.Stream(spec)
    ctx, orc = make_pair(spec.B, spec.H, spec.W, sky_mask=st.mask, pipeline_ingest=1)
    res = run_steps_sampled(ctx, orc, st.frame, list(range(spec.T)), label="streaming2048", tiles=1,
                            check_welford_at=(spec.T - 1,))
    assert res["steps"] == spec.T and res["zeta_checked"] > 0, res
    n_rfi = 0
    for t in range(spec.T):
        assert orc.rejected[t] & st.rfi_mask(t) == st.rfi_mask(t), t
        n_rfi += bin(st.rfi_mask(t)).count("1")
    assert n_rfi >= 5


@pytest.mark.parametrize("max_sources", [8192, 20000])
def test_many_peaks_catalogue_global_lists(max_sources):
    """More than 256 kept peaks and more than 240 peaks in one step (4 x
    1024^2 at kappa = 3.4, peak_cap 2048): the catalogue's candidate and
    neighbour lists leave the LDS for global memory, and with a table of
    20000 slots its taken / seen bitmaps too; events and spectra as the
    oracle's.  (More than 2048 peaks, which moves the sort keys, positions
    and flags to global memory, is the sweep test's kappa = 2 case.)"""
    _torch_cuda()
    rng = np.random.default_rng(44)
    B, H, W = 4, 1024, 1024
    ctx, orc = make_pair(B, H, W, kappa=3.4, peak_cap=2048, pipeline_ingest=1, max_sources=max_sources)

    def frame(t):
        return rng.standard_normal((B, H, W)).astype(np.float32)
    res = run_steps_sampled(ctx, orc, frame, [0, 1, 2], label=f"many-peaks-S{max_sources}", tiles=1)
    assert res["peaks"] / 3 > 1000, res
    assert ctx.status()["n_kept"] > 512
