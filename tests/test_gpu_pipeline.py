"""Pipelined ingest: with pipeline_ingest = 1 the next step's ingest and QC
run on a stream of the context's own, beside this step's catalogue and flux.
Every result must be bitwise the one of a sequential context: the kernels are
the same and the pipelining only reorders independent work."""

import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _stream(T):
    spec = synth.StreamSpec(
        name="pipe", B=8, H=192, W=192, T=T, freqs_mhz=synth.two_group_freqs(8),
        n_sources=6, amp=(12.0, 20.0), dm=(0.0, 60.0), width_choices=(1, 2), t0=(1.0, 9.0),
        integer_centres=False, mask=True, mask_shrink=24, min_sep=20.0, seed=321, cfg=5, stream=0)
    return synth.Stream(spec)


def _frames(st, T, rfi_at=9):
    out = []
    for t in range(T):
        f = st.frame(t).copy()
        if t == rfi_at:
            f[3] *= 5.0          # a whole band five times noisier: rejected by QC
        out.append(f)
    return out


PARAMS = dict(kappa=6.0, monitor_steps=4, backfill_steps=6)


def test_pipelined_ingest_same_results_per_step():
    torch = _torch_cuda()
    from paper_2103_15418_amd import Context
    T = 18
    st = _stream(T)
    frames = _frames(st, T)
    dev = [torch.from_numpy(f).cuda() for f in frames]
    torch.cuda.synchronize()
    seq = Context(8, 192, 192, sky_mask=st.mask, **PARAMS)
    pip = Context(8, 192, 192, sky_mask=st.mask, pipeline_ingest=1, **PARAMS)
    n_peaks = n_events = n_rej = 0
    for t in range(T):
        # host cubes on some steps exercise the copy on the ingest stream
        src = frames[t] if t % 5 == 2 else dev[t]
        r_seq = seq.ingest(t, src, want_rejected=True)
        r_pip = pip.ingest(t, src, want_rejected=(t % 2 == 0))
        if r_pip is not None:
            assert r_pip == r_seq, t
        n_rej += bin(r_seq).count("1")
        p_s, e_s, rc_s = seq.detect()
        p_p, e_p, rc_p = pip.detect()
        assert rc_s == rc_p and p_s.tobytes() == p_p.tobytes() and e_s.tobytes() == e_p.tobytes(), t
        n_peaks += len(p_s)
        n_events += len(e_s)
        seq.extract_flux()
        pip.extract_flux()
        for ev in e_s:
            if int(ev["event"]) == 2:      # ended: the dynamic spectra are the same
                a = seq.read_spectrum(int(ev["id"]))
                b = pip.read_spectrum(int(ev["id"]))
                assert a[0].tobytes() == b[0].tobytes() and (a[1] == b[1]).all() and a[2] == b[2], (t, ev)
        assert seq.status() == pip.status(), t
    assert n_peaks > 0 and n_events > 0 and n_rej > 0


def test_pipelined_ingest_asynchronous_steps():
    """Nothing synchronises between steps: detect without outputs, inference
    tickets collected one step late; the network's results, the final status
    and the cached planes equal the sequential context's."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Context, Model
    T = 22
    st = _stream(T)
    dev = [torch.from_numpy(f).cuda() for f in _frames(st, T)]
    torch.cuda.synchronize()
    wts = synth.cnn_weights(seed=3)

    def run(pipelined):
        ctx = Context(8, 192, 192, sky_mask=st.mask, pipeline_ingest=pipelined, **PARAMS)
        model = Model(wts, max_batch=32)
        pending, got = [], []
        for t in range(T):
            ctx.ingest(t, dev[t])
            ctx.detect(want=False)
            ctx.extract_flux()
            pending.append(model.infer_async([ctx]))
            if len(pending) > 1:
                got.append(model.collect(pending.pop(0)))
        while pending:
            got.append(model.collect(pending.pop(0)))
        planes = [ctx.debug_read(k).tobytes() for k in ("centre", "cache", "welford_mean", "welford_m2",
                                                         "welford_n", "bandstats")]
        return got, ctx.status(), planes

    g_seq, s_seq, p_seq = run(0)
    g_pip, s_pip, p_pip = run(1)
    assert s_seq == s_pip
    assert p_seq == p_pip
    n = 0
    for (mu_a, L_a, src_a), (mu_b, L_b, src_b) in zip(g_seq, g_pip):
        assert src_a.tobytes() == src_b.tobytes()
        assert mu_a.tobytes() == mu_b.tobytes() and L_a.tobytes() == L_b.tobytes()
        n += len(src_a)
    assert len(g_seq) == len(g_pip) == T and n > 0


def test_deferred_network_launch_flushed_by_destroy():
    """A pipelined context defers its ticket's network to its next detect; a
    ticket still deferred when the context is destroyed is launched then and
    stays collectible, with the sequential context's results."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Context, Model
    T = 13                      # episodes end at the last step
    st = _stream(T)
    dev = [torch.from_numpy(f).cuda() for f in _frames(st, T)]
    torch.cuda.synchronize()
    wts = synth.cnn_weights(seed=3)
    out = []
    for pipelined in (0, 1):
        ctx = Context(8, 192, 192, sky_mask=st.mask, pipeline_ingest=pipelined, **PARAMS)
        model = Model(wts, max_batch=32)
        for t in range(T):
            ctx.ingest(t, dev[t])
            ctx.detect(want=False)
            ctx.extract_flux()
        tk = model.infer_async([ctx])
        ctx.__del__()           # lpf_destroy with the launch still deferred
        out.append(model.collect(tk))
    (mu_a, L_a, src_a), (mu_b, L_b, src_b) = out
    assert len(src_a) > 0
    assert src_a.tobytes() == src_b.tobytes()
    assert mu_a.tobytes() == mu_b.tobytes() and L_a.tobytes() == L_b.tobytes()


def test_model_destroyed_with_deferred_ticket():
    """A model destroyed while a pipelined context still holds its deferred
    ticket: the context goes on (its next detect launches nothing of the
    model) and a new model's results equal the sequential context's."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Context, Model
    T = 16
    st = _stream(T)
    dev = [torch.from_numpy(f).cuda() for f in _frames(st, T)]
    torch.cuda.synchronize()
    wts = synth.cnn_weights(seed=3)
    out = []
    for pipelined in (0, 1):
        ctx = Context(8, 192, 192, sky_mask=st.mask, pipeline_ingest=pipelined, **PARAMS)
        for t in range(12):
            ctx.ingest(t, dev[t])
            ctx.detect(want=False)
            ctx.extract_flux()
        doomed = Model(wts, max_batch=32)
        doomed.infer_async([ctx])
        doomed.__del__()        # lpf_model_destroy with the ticket deferred
        for t in range(12, T):
            ctx.ingest(t, dev[t])
            ctx.detect(want=False)
            ctx.extract_flux()
        model = Model(wts, max_batch=32)
        out.append((model.collect(model.infer_async([ctx])), ctx.status()))
    (r_a, s_a), (r_b, s_b) = out
    assert s_a == s_b
    for x, y in zip(r_a, r_b):
        assert x.tobytes() == y.tobytes()


def test_pipelined_ingest_with_gaps_in_t():
    """Time stamps that skip steps (gaps of 2 and 3): the frame after a gap
    overwrites the cache slot the backfill of the flux just enqueued may
    read, so that ingest waits for the whole previous step.  Every source's
    dynamic spectrum (backfilled ones included) and the status equal the
    sequential context's."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Context
    ts = [0, 1, 2, 4, 5, 6, 9, 10, 12, 13, 14, 15, 18, 19, 20, 21]
    st = _stream(max(ts) + 1)
    frames = _frames(st, max(ts) + 1, rfi_at=-1)
    dev = {t: torch.from_numpy(frames[t]).cuda() for t in ts}
    torch.cuda.synchronize()
    seq = Context(8, 192, 192, sky_mask=st.mask, **PARAMS)
    pip = Context(8, 192, 192, sky_mask=st.mask, pipeline_ingest=1, **PARAMS)
    ids = set()
    for t in ts:
        for c in (seq, pip):
            c.ingest(t, dev[t])
        _, e_s, _ = seq.detect()
        _, e_p, _ = pip.detect()
        assert e_s.tobytes() == e_p.tobytes(), t
        ids |= {int(ev["id"]) for ev in e_s}
        seq.extract_flux()
        pip.extract_flux()
    assert seq.status() == pip.status()
    from paper_2103_15418_amd._abi import LpfError

    def spectrum(c, sid):
        try:
            return c.read_spectrum(sid)
        except LpfError:
            return None   # released after its monitoring window
    n = 0
    for sid in sorted(ids):
        a, b = spectrum(seq, sid), spectrum(pip, sid)
        assert (a is None) == (b is None), sid
        if a is not None:
            assert a[0].tobytes() == b[0].tobytes() and (a[1] == b[1]).all() and a[2] == b[2], sid
            n += 1
    assert n > 0, ids
