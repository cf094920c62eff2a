"""Batch calls (lpf_ingest_batch / lpf_detect_batch / lpf_extract_flux_batch):
grouped launches over contexts of uneven B, H and W give bitwise the results
of the per-context calls on every step: QC statistics, peaks, events,
counters, the centre plane, dynamic spectra and the pooled network outputs.

The mix is the serving workload's eight streams (2 x 512^2, 2 x 1024^2,
2 x 2048^2 with 16 bands, 2 x 1536^2 with 8 bands) plus two contexts whose
filters cannot join a group (two clip iterations; a width that is not a
multiple of 4), ten contexts in all, so the calls also split into groups of
at most eight."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _specs(T):
    specs = synth.spec_serving_streams(T=T)
    for s in specs:
        s.t0 = (0.0, 4.0)
        s.dm = (0.0, 60.0)      # most sweeps fall inside the run
    extra = [
        synth.StreamSpec(name="clip2", B=16, H=256, W=256, T=T, freqs_mhz=synth.two_group_freqs(16), n_sources=4,
                         amp=(10.0, 20.0), dm=(0.0, 40.0), t0=(0.0, 4.0), integer_centres=False, mask=True,
                         mask_shrink=30, seed=91, cfg=5, stream=8),
        synth.StreamSpec(name="w250", B=4, H=200, W=250, T=T, freqs_mhz=np.linspace(60.0, 70.0, 4), n_sources=3,
                         amp=(10.0, 20.0), dm=(0.0, 40.0), t0=(0.0, 4.0), integer_centres=True,
                         place_box=(30, 170), seed=92, cfg=5, stream=9),
    ]
    return specs + extra


PARAMS = dict(monitor_steps=4, backfill_steps=6)


def test_batch_calls_bitwise_equal_per_context_calls():
    torch = _torch_cuda()
    import paper_2103_15418_amd as P
    T = 12
    specs = _specs(T)
    streams = [synth.Stream(s) for s in specs]
    extra = {"clip2": dict(clip_iters=2)}
    mk = lambda st: P.Context(st.spec.B, st.spec.H, st.spec.W, sky_mask=st.mask if st.spec.mask else None,
                              **PARAMS, **extra.get(st.spec.name, {}))
    cb = [mk(st) for st in streams]
    cr = [mk(st) for st in streams]
    model = P.Model(synth.cnn_weights(), max_batch=256)
    n_ended = n_spec = n_peaks = 0
    for t in range(T):
        print(f"batch step t={t}", flush=True)
        cubes = [torch.from_numpy(st.frame(t)).cuda() for st in streams]
        P.ingest_batch(cb, [t] * len(cb), cubes)
        P.detect_batch(cb)
        P.extract_flux_batch(cb)
        for c, cube in zip(cr, cubes):
            c.ingest(t, cube)
            c.detect(want=False)
            c.extract_flux()
        for k, (a, b) in enumerate(zip(cb, cr)):
            sa, sb = a.status(), b.status()
            assert sa == sb, (t, specs[k].name, sa, sb)
            pa, ea = a.last_lists()
            pb, eb = b.last_lists()
            assert pa.tobytes() == pb.tobytes(), (t, specs[k].name)
            assert ea.tobytes() == eb.tobytes(), (t, specs[k].name)
            assert np.array_equal(a.debug_read("bandstats"), b.debug_read("bandstats")), (t, k)
            if t % 4 == 3:
                assert np.array_equal(a.debug_read("centre"), b.debug_read("centre")), (t, k)
            n_peaks += len(pa)
            for sid in sorted({int(e["id"]) for e in ea} | {int(e["id"]) for e in eb}):
                if any(int(e["id"]) == sid and int(e["event"]) == P.EVENT_ENDED for e in ea):
                    continue   # an ended episode's record is released at the next step
                oa = a.read_spectrum(sid)
                ob = b.read_spectrum(sid)
                assert np.array_equal(oa[0], ob[0]) and np.array_equal(oa[1], ob[1]) and oa[2] == ob[2], (t, k, sid)
                n_spec += 1
        mu_a, L_a, s_a = model.infer(cb)
        mu_b, L_b, s_b = model.infer(cr)
        assert np.array_equal(s_a, s_b) and np.array_equal(mu_a, mu_b) and np.array_equal(L_a, L_b), t
        n_ended += len(s_a)
    print(f"batch: peaks {n_peaks}, spectra compared {n_spec}, ended episodes inferred {n_ended}", flush=True)
    assert n_peaks > 50 and n_spec > 20 and n_ended > 0


def test_batch_call_checks():
    """Contexts on different streams, pipelined contexts, repeated contexts and
    call-order violations are refused before anything runs."""
    torch = _torch_cuda()
    import paper_2103_15418_amd as P
    from paper_2103_15418_amd import LpfError
    a = P.Context(4, 64, 64)
    b = P.Context(4, 64, 64)
    s = torch.cuda.Stream()
    c = P.Context(4, 64, 64, stream=s)
    d = P.Context(4, 64, 64, pipeline_ingest=1)
    cube = torch.zeros((4, 64, 64), device="cuda")
    for bad, code in (([a, c], P.LPF_EINVAL), ([a, d], P.LPF_EINVAL), ([a, a], P.LPF_EINVAL)):
        with pytest.raises(LpfError) as err:
            P.ingest_batch(bad, [0] * len(bad), [cube] * len(bad))
        assert err.value.code == code
    with pytest.raises(LpfError) as err:
        P.detect_batch([a, b])
    assert err.value.code == -6   # LPF_ESTATE: no ingest yet
    P.ingest_batch([a, b], [0, 0], [cube, cube])
    with pytest.raises(LpfError) as err:
        P.ingest_batch([a, b], [1, 1], [cube, cube])
    assert err.value.code == -6
    P.detect_batch([a, b])
    P.extract_flux_batch([a, b])
    with pytest.raises(LpfError) as err:
        P.ingest_batch([a, b], [1, 0], [cube, cube])
    assert err.value.code == -4   # LPF_EORDER for b; nothing ran for a
    P.ingest_batch([a, b], [1, 1], [cube, cube])
    torch.cuda.synchronize()
