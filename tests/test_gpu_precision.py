"""Precision form: filters and network with bf16 / fp16 operands on MFMA and
float32 accumulation, against the FP64 oracle.

There is no parity gate for 16-bit arithmetic; the tests print the error per
output (max and median, relative to the same condition scales as the FP32
tests) and check loose bounds derived from the unit roundoff
(bf16 u = 2^-8, fp16 u = 2^-11, a few roundings per output):
filters |err| <= 8u * scale, network |err| <= 16u * scale; and that the 16-bit
candidate lists agree with FP32 except where the oracle's sig lies within
that filter bound, carried to sig, of the threshold.
"""

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
from oracle.filters import centre_spread, correlate_2d

from parity import cnn_scale, make_pair, oracle_sig_map

pytestmark = pytest.mark.gpu

U = {1: 2.0 ** -8, 2: 2.0 ** -11}   # unit roundoff by precision code
NAME = {1: "bf16", 2: "fp16"}


def _torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("prec", [1, 2])
def test_filter_planes_16bit_error(prec):
    _torch_cuda()
    spec = synth.spec_instrument(T=1, H=512)
    spec.n_sources = 20
    st = synth.Stream(spec)
    ctx, orc = make_pair(spec.B, spec.H, spec.W, sky_mask=st.mask, debug_planes=1,
                         filter_precision=prec)
    cube = st.frame(0)
    orc.ingest(0, cube)
    ctx.ingest(0, cube)
    orc.detect()
    ctx.detect()
    Cd, Sd = ctx.debug_read("centre"), ctx.debug_read("spread")
    M, g = orc.M, orc.g
    worst_c = worst_s = 0.0
    med_c, med_s = [], []
    for b in range(0, spec.B, 4):
        X = cube[b]
        C, S, den = centre_spread(X, M, g)
        pos = (den > 0) & M
        safe = np.where(den > 0, den, 1.0)
        scC = (correlate_2d(M * np.abs(X.astype(np.float64)), g) / safe)[pos]
        scS = (correlate_2d(M * (np.abs(X.astype(np.float64)) + np.abs(C)) ** 2, g) / safe)[pos]
        assert np.isfinite(Cd[b][pos]).all() and np.isfinite(Sd[b][pos]).all(), (NAME[prec], b)
        rc = np.abs(Cd[b][pos] - C[pos]) / scC
        rs = np.abs(Sd[b][pos] - S[pos]) / scS
        worst_c, worst_s = max(worst_c, float(np.max(rc))), max(worst_s, float(np.max(rs)))
        med_c.append(np.median(rc))
        med_s.append(np.median(rs))
    print(f"{NAME[prec]} filter error / scale: C max {worst_c:.2e} median {np.median(med_c):.2e}; "
          f"S max {worst_s:.2e} median {np.median(med_s):.2e}", flush=True)
    assert worst_c <= 8 * U[prec] and worst_s <= 8 * U[prec]


@pytest.mark.parametrize("prec", [1, 2])
def test_candidates_16bit_vs_fp32(prec):
    """Peak lists of the 16-bit filters against the FP32 path on the instrument
    workload: differences only where the oracle's sig is within the 16-bit
    error of the threshold; Jaccard index reported."""
    _torch_cuda()
    spec = synth.spec_instrument(T=3)
    st = synth.Stream(spec)
    from paper_2103_15418_amd import Context
    c32 = Context(spec.B, spec.H, spec.W, sky_mask=st.mask)
    c16 = Context(spec.B, spec.H, spec.W, sky_mask=st.mask, filter_precision=prec)
    inter = union = 0
    far = 0
    for t in range(spec.T):
        cube = st.frame(t)
        c32.ingest(t, cube)
        c16.ingest(t, cube)
        p32 = {(int(p["band"]), int(p["row"]), int(p["col"])) for p in c32.detect()[0]}
        p16 = {(int(p["band"]), int(p["row"]), int(p["col"])) for p in c16.detect()[0]}
        c32.extract_flux()
        c16.extract_flux()
        inter += len(p32 & p16)
        union += len(p32 | p16)
        diff = p32 ^ p16
        if diff:
            from oracle.filters import taps_1d
            g = taps_1d(0, 8.0, 24)
            M = st.mask.astype(bool)
            den = correlate_2d(M.astype(np.float64), g)
            maps = {}
            for (b, i, j) in sorted(diff):
                # the filters' error bound (8u of the scales, as gated above)
                # carried to sig = (x - c)/sqrt(s):
                #   |d sig| <= 8u (scC / sqrt(S) + |sig| scS / (2 S))
                if b not in maps:
                    Q, sig, C, S = oracle_sig_map(cube[b], M, g, 3)
                    xa = np.abs(cube[b].astype(np.float64))
                    maps[b] = (sig, S, correlate_2d(M * xa, g) / den, correlate_2d(M * (xa + np.abs(C)) ** 2, g) / den)
                sig, S, scC, scS = maps[b]
                bound = 8 * U[prec] * (scC[i, j] / np.sqrt(S[i, j]) + abs(sig[i, j]) * scS[i, j] / (2 * S[i, j]))
                if abs(sig[i, j] - 4.5) > bound:
                    far += 1
    jac = inter / max(1, union)
    print(f"{NAME[prec]} candidates vs fp32: Jaccard {jac:.4f} ({inter}/{union}), far differences {far}",
          flush=True)
    assert far == 0 and jac >= 0.9


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("n,maxb", [(70, 64), (300, 512)])
def test_network_16bit_error(prec, n, maxb):
    """70 windows through a model of batch 64 (two chunks, the per-32-window
    fc1), 300 through one of batch 512 (one call: the fc1 over 128-window
    blocks, the last one ragged)."""
    torch = _torch_cuda()
    from paper_2103_15418_amd import Model
    wts = synth.cnn_weights(seed=11)
    rng = np.random.default_rng(4)
    x = (rng.standard_normal((n, 16, 64)) * 2.0).astype(np.float32)
    x[::3, 5, 20:30] += 6.0
    m = Model(wts, precision=prec, max_batch=maxb)
    mu_d, L_d = m.infer_windows(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    raw = ocnn.forward_raw(x.astype(np.float64), wts)
    mu_o, L_o = ocnn.head(raw)
    sc = cnn_scale(x.astype(np.float64), wts)
    err = np.concatenate([np.abs(mu_d.cpu().numpy() - mu_o) / sc[:, :4],
                          np.abs(L_d.cpu().numpy() - L_o) / sc[:, 4:]], axis=1)
    names = ["mu_DM", "mu_w", "mu_A", "mu_t"] + [f"L{k}" for k in range(10)]
    line = ", ".join(f"{n} {err[:, i].max():.1e}/{np.median(err[:, i]):.1e}" for i, n in enumerate(names))
    print(f"{NAME[prec]} network error / scale (max/median): {line}", flush=True)
    assert err.max() <= 16 * U[prec]
