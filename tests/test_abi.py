"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/lpf.h, and validates configurations without a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lpf_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_four_stages():
    names = declared_functions()
    for n in ("lpf_ingest_frame", "lpf_detect", "lpf_extract_flux", "lpf_infer"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2103_15418_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    lib = C.CDLL(P.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_config_validation_host_only():
    import paper_2103_15418_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    cfg = P.default_config(16, 1024, 1024)
    n = P.workspace_size(cfg)
    # cache (33 cubes) + Welford (4 planes) + centre dominate: > 37 planes of 64 MiB
    assert n > 37 * 64 * 2 ** 20
    for bad in (dict(B=17), dict(B=0), dict(H=5000), dict(ring_len=32), dict(clip_iters=0),
                dict(peak_cap=600), dict(bg_halfwidth=41), dict(filter_precision=3),
                dict(filter_precision=1, clip_iters=2), dict(filter_precision=2, bg_halfwidth=10),
                dict(max_sources=0), dict(peak_halfwidth=0), dict(pipeline_ingest=2),
                dict(pipeline_ingest=-1), dict(kappa=-1.0)):
        c = P.default_config(16, 1024, 1024)
        for k, v in bad.items():
            setattr(c, k, v)
        with pytest.raises(P.LpfError):
            P.workspace_size(c)


def test_weights_blob_size_and_packing():
    import numpy as np

    import paper_2103_15418_amd as P
    import synth
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    wts = synth.cnn_weights(seed=1)
    blob = P.pack_weights(wts)
    assert len(blob) == P.lib().lpf_model_weights_bytes()
    arr = np.frombuffer(blob, dtype=np.float32)
    assert arr[0] == wts["conv1.w"].ravel()[0] and arr[-1] == 0.0
    bad = dict(wts)
    bad["fc2.b"] = np.zeros(13, dtype=np.float32)
    with pytest.raises(ValueError):
        P.pack_weights(bad)


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2103_15418_amd._abi as A
    monkeypatch.setattr(A, "_lib", None)
    monkeypatch.setattr(A, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        A.lib()


def test_pipelined_ingest_holds_one_cube_more():
    """With the pipelined ingest the image cache holds backfill + 2 cubes (the
    next step is written while this one is measured): exactly one cube more,
    plus one more step of the cutout staging (B x 65^2 floats)."""
    import paper_2103_15418_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    for B, H, W in ((16, 1024, 1024), (4, 96, 80)):
        seq = P.workspace_size(P.default_config(B, H, W))
        pip = P.workspace_size(P.default_config(B, H, W, pipeline_ingest=1))
        cube = B * H * W * 4
        assert cube <= pip - seq <= cube + B * 65 * 65 * 4 + 512


def test_select_candidates_matches_oracle():
    """Host-only selection (no device call): DM cut, sigma_DM cut and order
    against the oracle's selection, with ties and values on both cut edges."""
    import numpy as np
    import paper_2103_15418_amd as P
    from oracle.alert import select
    rng = np.random.default_rng(5)
    n = 300
    mu = rng.uniform(0, 200, (n, 4)).astype(np.float32)
    L = rng.uniform(-3, 3, (n, 10)).astype(np.float32)
    L[:, 0] = rng.choice([1.0, 2.5, 50.0, 60.0, 10.0, 49.999996], n).astype(np.float32)
    mu[::7, 0] = 50.0
    idx, sg = P.select_candidates(mu, L, 50.0, 50.0)
    ref, sref = select(mu, L, 50.0, 50.0)
    assert list(idx) == list(ref)
    assert np.array_equal(sg.astype(np.float64), sref)
    idx0, _ = P.select_candidates(mu[:0], L[:0])
    assert len(idx0) == 0
