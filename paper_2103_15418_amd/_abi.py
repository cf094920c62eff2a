"""ctypes binding of liblpf (include/lpf.h): argument marshalling only.

Every step of the pipeline runs in the HIP library; this module only
allocates workspaces as torch tensors, passes pointers and the current torch
stream, and converts host results to numpy.  It raises if the library is
missing instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpf.so")

LPF_OK, LPF_EINVAL, LPF_ENOMEM, LPF_EFULL, LPF_EORDER, LPF_EDEVICE, LPF_ESTATE = 0, -1, -2, -3, -4, -5, -6
KERNEL_GAUSS, KERNEL_BOX, KERNEL_DISK = 0, 1, 2
PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
EVENT_NEW, EVENT_ENDED = 1, 2
DBG = dict(bandstats=1, welford_mean=2, welford_m2=3, welford_n=4, centre=5, spread=6,
           clipmask=7, cache=8, peaks=9, events=10, prefiltered=11)
_ERRNAMES = {LPF_EINVAL: "EINVAL", LPF_ENOMEM: "ENOMEM", LPF_EFULL: "EFULL",
             LPF_EORDER: "EORDER", LPF_EDEVICE: "EDEVICE", LPF_ESTATE: "ESTATE"}


class LpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lpf error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("B", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
        ("sky_mask", C.c_void_p), ("grid_rows", C.c_void_p),
        ("kappa", C.c_float), ("bg_sigma", C.c_float), ("bg_halfwidth", C.c_int32),
        ("kernel", C.c_int32), ("clip_iters", C.c_int32), ("peak_halfwidth", C.c_int32),
        ("flux_halfwidth", C.c_int32), ("dup_radius", C.c_float), ("assoc_radius", C.c_float),
        ("monitor_steps", C.c_int32), ("backfill_steps", C.c_int32), ("ring_len", C.c_int32),
        ("qc_band_z", C.c_float), ("qc_rms_z", C.c_float), ("qc_rms_floor", C.c_float),
        ("qc_pixel_zeta", C.c_float), ("qc_warmup", C.c_int32), ("max_sources", C.c_int32),
        ("peak_cap", C.c_int32), ("filter_precision", C.c_int32), ("debug_planes", C.c_int32),
        ("pipeline_ingest", C.c_int32), ("psf_sigma", C.c_float), ("psf_halfwidth", C.c_int32),
        ("flux_bg_width", C.c_int32),
    ]


class Peak(C.Structure):
    _fields_ = [("band", C.c_int32), ("row", C.c_int32), ("col", C.c_int32),
                ("x", C.c_float), ("c", C.c_float), ("s", C.c_float), ("sig", C.c_float)]


class Source(C.Structure):
    _fields_ = [("id", C.c_int32), ("row", C.c_int32), ("col", C.c_int32), ("event", C.c_int32),
                ("t_first", C.c_int64), ("t_last_det", C.c_int64), ("t_end", C.c_int64)]


class Status(C.Structure):
    _fields_ = [("t", C.c_int64), ("rejected_bands", C.c_uint32), ("overflow_bands", C.c_uint32),
                ("n_peaks", C.c_int32), ("n_kept", C.c_int32), ("n_new", C.c_int32),
                ("n_ended", C.c_int32), ("n_measured", C.c_int32), ("n_dropped", C.c_int32),
                ("n_live", C.c_int32)]


PEAK_DTYPE = np.dtype([("band", "<i4"), ("row", "<i4"), ("col", "<i4"), ("x", "<f4"),
                       ("c", "<f4"), ("s", "<f4"), ("sig", "<f4")])
SOURCE_DTYPE = np.dtype([("id", "<i4"), ("row", "<i4"), ("col", "<i4"), ("event", "<i4"),
                         ("t_first", "<i8"), ("t_last_det", "<i8"), ("t_end", "<i8")])

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liblpf.so not built at {LIB_PATH}; run python -m paper_2103_15418_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "lpf_config_default": (i32, [C.POINTER(Config), i32, i32, i32]),
        "lpf_workspace_size": (i32, [C.POINTER(Config), C.POINTER(sz)]),
        "lpf_create": (i32, [C.POINTER(Config), vp, sz, vp, C.POINTER(vp)]),
        "lpf_destroy": (None, [vp]),
        "lpf_ingest_frame": (i32, [vp, i64, vp, i32, C.POINTER(C.c_uint32)]),
        "lpf_detect": (i32, [vp, vp, i32, C.POINTER(i32), vp, i32, C.POINTER(i32)]),
        "lpf_extract_flux": (i32, [vp]),
        "lpf_ingest_batch": (i32, [vp, vp, vp, i32, i32]),
        "lpf_detect_batch": (i32, [vp, i32]),
        "lpf_extract_flux_batch": (i32, [vp, i32]),
        "lpf_status": (i32, [vp, C.POINTER(Status)]),
        "lpf_read_spectrum": (i32, [vp, i32, vp, vp, C.POINTER(i64)]),
        "lpf_model_weights_bytes": (sz, []),
        "lpf_model_workspace_size": (i32, [i32, i32, C.POINTER(sz)]),
        "lpf_model_create": (i32, [vp, sz, i32, i32, vp, sz, vp, C.POINTER(vp)]),
        "lpf_model_destroy": (None, [vp]),
        "lpf_infer": (i32, [vp, i32, vp, vp, i32, vp, vp, vp, i32, C.POINTER(i32)]),
        "lpf_infer_async": (i32, [vp, i32, vp, C.POINTER(C.c_int64)]),
        "lpf_infer_collect": (i32, [vp, C.c_int64, vp, vp, vp, i32, C.POINTER(i32)]),
        "lpf_infer_windows": (i32, [vp, vp, i32, vp, vp, vp]),
        "lpf_infer_windows_static": (i32, [vp, vp, i32, vp, vp, vp]),
        "lpf_debug_read": (i32, [vp, i32, vp, sz]),
        "lpf_select_candidates": (i32, [vp, vp, i32, C.c_float, C.c_float, vp, vp, C.POINTER(i32)]),
        "lpf_read_cutouts": (i32, [vp, i32, i32, i32, i64, i32, vp, vp]),
        "lpf_checkpoint_size": (i32, [vp, C.POINTER(sz)]),
        "lpf_checkpoint_save": (i32, [vp, vp, sz]),
        "lpf_checkpoint_load": (i32, [vp, vp, sz]),
        "lpf_sync": (i32, [vp]),
        "lpf_profile_enable": (i32, [vp, i32]),
        "lpf_profile_read": (i32, [vp, vp, vp]),
        "lpf_last_error": (C.c_char_p, [vp]),
        "lpf_server_create": (i32, [vp, sz, i32, C.POINTER(vp)]),
        "lpf_server_destroy": (None, [vp]),
        "lpf_server_admit": (i32, [vp, C.POINTER(Config), vp, sz, i32, C.POINTER(i32), C.POINTER(i32)]),
        "lpf_server_close": (i32, [vp, i32]),
        "lpf_server_submit": (i32, [vp, i32, i64, vp, i32, i64]),
        "lpf_server_poll": (i32, [vp, vp, i32, C.POINTER(i32)]),
        "lpf_server_drain": (i32, [vp]),
        "lpf_server_fetch": (i32, [vp, i32, i64, vp, i32, C.POINTER(i32), vp, i32, C.POINTER(i32),
                                   vp, vp, vp, i32, C.POINTER(i32)]),
        "lpf_server_usage": (i32, [vp, C.POINTER(sz), C.POINTER(sz), C.POINTER(i32)]),
        "lpf_now_ns": (i64, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _torch():
    import torch
    return torch


def default_config(B: int, H: int, W: int, **kw) -> Config:
    cfg = Config()
    rc = lib().lpf_config_default(C.byref(cfg), B, H, W)
    if rc != LPF_OK:
        raise LpfError(rc, "config_default")
    for k, v in kw.items():
        if not hasattr(cfg, k) or k in ("sky_mask", "grid_rows"):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def workspace_size(cfg: Config) -> int:
    n = C.c_size_t(0)
    rc = lib().lpf_workspace_size(C.byref(cfg), C.byref(n))
    if rc != LPF_OK:
        raise LpfError(rc, "invalid configuration")
    return int(n.value)


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Context:
    """One image stream: workspace (a torch uint8 tensor) + library context."""

    def __init__(self, B: int, H: int, W: int, sky_mask: Optional[np.ndarray] = None,
                 grid_rows: Optional[Sequence[int]] = None, device: str = "cuda:0",
                 stream=None, **params):
        torch = _torch()
        self.B, self.H, self.W = B, H, W
        self.cfg = default_config(B, H, W, **params)
        self._mask = None
        if sky_mask is not None:
            self._mask = np.ascontiguousarray(sky_mask, dtype=np.uint8)
            assert self._mask.shape == (H, W)
            self.cfg.sky_mask = self._mask.ctypes.data
        self._rows = None
        if grid_rows is not None:
            self._rows = np.ascontiguousarray(grid_rows, dtype=np.int32)
            self.cfg.grid_rows = self._rows.ctypes.data
        self.ws_bytes = workspace_size(self.cfg)
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream
        h = C.c_void_p()
        rc = lib().lpf_create(C.byref(self.cfg), C.c_void_p(self.workspace.data_ptr()),
                              self.ws_bytes, C.c_void_p(_stream_ptr(stream)), C.byref(h))
        self.cfg.sky_mask = None
        self.cfg.grid_rows = None
        if rc != LPF_OK:
            raise LpfError(rc, "lpf_create failed")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.lpf_destroy(h)
            self.h = None

    def _check(self, rc: int, what: str, allow=()):
        if rc != LPF_OK and rc not in allow:
            raise LpfError(rc, f"{what}: {lib().lpf_last_error(self.h).decode()}")
        return rc

    # -- the four stages -----------------------------------------------------------
    def ingest(self, t: int, cube, want_rejected: bool = False) -> Optional[int]:
        torch = _torch()
        if isinstance(cube, torch.Tensor):
            # device tensor, or host tensor (pinned memory keeps the copy asynchronous)
            assert cube.dtype == torch.float32 and cube.is_contiguous()
            assert tuple(cube.shape) == (self.B, self.H, self.W)
            ptr, on_dev = cube.data_ptr(), (1 if cube.is_cuda else 0)
            keep = cube
        else:
            keep = np.ascontiguousarray(cube, dtype=np.float32)
            assert keep.shape == (self.B, self.H, self.W)
            ptr, on_dev = keep.ctypes.data, 0
        rej = C.c_uint32(0)
        self._check(lib().lpf_ingest_frame(self.h, int(t), C.c_void_p(ptr), on_dev,
                                           C.byref(rej) if want_rejected else None), "ingest")
        del keep
        return int(rej.value) if want_rejected else None

    def detect(self, want: bool = True):
        """Returns (peaks structured array, events structured array, rc) or None."""
        if not want:
            self._check(lib().lpf_detect(self.h, None, 0, None, None, 0, None), "detect")
            return None
        cap = self.B * self.cfg.peak_cap
        peaks = np.zeros(cap, dtype=PEAK_DTYPE)
        ev_cap = 2 * self.cfg.max_sources
        events = np.zeros(ev_cap, dtype=SOURCE_DTYPE)
        n_p, n_e = C.c_int32(0), C.c_int32(0)
        rc = self._check(lib().lpf_detect(self.h, C.c_void_p(peaks.ctypes.data), cap, C.byref(n_p),
                                          C.c_void_p(events.ctypes.data), ev_cap, C.byref(n_e)),
                         "detect", allow=(LPF_EFULL,))
        return peaks[:min(cap, n_p.value)].copy(), events[:min(ev_cap, n_e.value)].copy(), rc

    def extract_flux(self):
        self._check(lib().lpf_extract_flux(self.h), "extract_flux")

    def status(self) -> Dict[str, int]:
        st = Status()
        self._check(lib().lpf_status(self.h, C.byref(st)), "status")
        return {k: int(getattr(st, k)) for k, _ in Status._fields_}

    def read_spectrum(self, sid: int):
        out = np.zeros((self.B, 64), dtype=np.float32)
        valid = np.zeros((self.B, 64), dtype=np.uint8)
        tl = C.c_int64(0)
        self._check(lib().lpf_read_spectrum(self.h, int(sid), C.c_void_p(out.ctypes.data),
                                            C.c_void_p(valid.ctypes.data), C.byref(tl)), "read_spectrum")
        return out, valid.astype(bool), int(tl.value)

    def debug_read(self, what: str) -> np.ndarray:
        B, H, W = self.B, self.H, self.W
        shape, dt = {
            "bandstats": ((B, 6), np.float64), "welford_mean": ((B, H, W), np.float32),
            "welford_m2": ((B, H, W), np.float32), "welford_n": ((B,), np.int32),
            "centre": ((B, H, W), np.float32), "spread": ((B, H, W), np.float32),
            "clipmask": ((B, H, W), np.uint8), "cache": ((B, H, W), np.float32),
            "prefiltered": ((B, H, W), np.float32)}[what]
        out = np.zeros(shape, dtype=dt)
        self._check(lib().lpf_debug_read(self.h, DBG[what], C.c_void_p(out.ctypes.data), out.nbytes),
                    f"debug_read({what})")
        return out

    def last_lists(self):
        """Peaks and raw events of the last detect, read from the device
        (for calls that returned nothing, e.g. the batch forms)."""
        st = self.status()
        peaks = np.zeros(st["n_peaks"], dtype=PEAK_DTYPE)
        events = np.zeros(st["n_new"] + st["n_ended"], dtype=SOURCE_DTYPE)
        self._check(lib().lpf_debug_read(self.h, DBG["peaks"], C.c_void_p(peaks.ctypes.data), peaks.nbytes),
                    "debug_read(peaks)")
        self._check(lib().lpf_debug_read(self.h, DBG["events"], C.c_void_p(events.ctypes.data), events.nbytes),
                    "debug_read(events)")
        return peaks, events

    def read_cutouts(self, row: int, col: int, half: int, t_first: int, n_steps: int):
        """[n_steps][B][2h+1][2h+1] boxes of the cached cubes and the cached flags."""
        side = 2 * half + 1
        out = np.zeros((n_steps, self.B, side, side), dtype=np.float32)
        have = np.zeros(n_steps, dtype=np.uint8)
        self._check(lib().lpf_read_cutouts(self.h, int(row), int(col), int(half), int(t_first), int(n_steps),
                                           C.c_void_p(out.ctypes.data), C.c_void_p(have.ctypes.data)),
                    "read_cutouts")
        return out, have.astype(bool)

    def checkpoint(self) -> np.ndarray:
        """The context's state between steps as a uint8 array."""
        n = C.c_size_t(0)
        self._check(lib().lpf_checkpoint_size(self.h, C.byref(n)), "checkpoint_size")
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(lib().lpf_checkpoint_save(self.h, C.c_void_p(buf.ctypes.data), buf.nbytes), "checkpoint_save")
        return buf

    def restore(self, buf: np.ndarray) -> None:
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(lib().lpf_checkpoint_load(self.h, C.c_void_p(buf.ctypes.data), buf.nbytes), "checkpoint_load")

    def sync(self):
        self._check(lib().lpf_sync(self.h), "sync")

    STAGES = ("ingest", "qc_decide", "centre", "spread_peaks", "catalog", "flux", "network")

    def profile(self, on: bool = True, stages: Optional[Sequence[str]] = None):
        """Time every stage (on=True), the named stages only, or none (on=False)."""
        mask = 0
        if on:
            mask = (1 << len(self.STAGES)) - 1 if stages is None else \
                sum(1 << self.STAGES.index(k) for k in stages)
        self._check(lib().lpf_profile_enable(self.h, mask), "profile_enable")

    def profile_read(self):
        """{stage: (total ms, launches)} since the last read."""
        ms = np.zeros(len(self.STAGES), dtype=np.float64)
        cnt = np.zeros(len(self.STAGES), dtype=np.int64)
        self._check(lib().lpf_profile_read(self.h, C.c_void_p(ms.ctypes.data),
                                           C.c_void_p(cnt.ctypes.data)), "profile_read")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.STAGES)}


def select_candidates(mu: np.ndarray, L: np.ndarray, dm_min: float = 50.0, sigma_max: float = 50.0):
    """lpf_select_candidates: (row indices ordered by sigma_DM, sigma_DM of every row)."""
    mu = np.ascontiguousarray(mu, dtype=np.float32)
    L = np.ascontiguousarray(L, dtype=np.float32)
    n = len(mu)
    idx = np.zeros(max(n, 1), dtype=np.int32)
    sg = np.zeros(max(n, 1), dtype=np.float32)
    k = C.c_int32(0)
    rc = lib().lpf_select_candidates(C.c_void_p(mu.ctypes.data), C.c_void_p(L.ctypes.data), n, float(dm_min),
                                     float(sigma_max), C.c_void_p(idx.ctypes.data), C.c_void_p(sg.ctypes.data),
                                     C.byref(k))
    if rc != LPF_OK:
        raise LpfError(rc, "select_candidates")
    return idx[:k.value].copy(), sg[:n].copy()


def _ctx_array(ctxs: Sequence["Context"]):
    return (C.c_void_p * len(ctxs))(*[c.h for c in ctxs])


def _batch_check(ctxs, rc: int, what: str):
    if rc != LPF_OK:
        msgs = "; ".join(lib().lpf_last_error(c.h).decode() for c in ctxs if lib().lpf_last_error(c.h))
        raise LpfError(rc, f"{what}: {msgs}")


def ingest_batch(ctxs: Sequence["Context"], ts: Sequence[int], cubes: Sequence) -> None:
    """lpf_ingest_batch: one cube per context, all torch CUDA tensors or all host arrays."""
    torch = _torch()
    holders, ptrs = [], []
    on_dev = None
    for c, cube in zip(ctxs, cubes):
        if isinstance(cube, torch.Tensor):
            assert cube.dtype == torch.float32 and cube.is_contiguous()
            assert tuple(cube.shape) == (c.B, c.H, c.W)
            dev = 1 if cube.is_cuda else 0
            holders.append(cube)
            ptrs.append(cube.data_ptr())
        else:
            a = np.ascontiguousarray(cube, dtype=np.float32)
            assert a.shape == (c.B, c.H, c.W)
            dev = 0
            holders.append(a)
            ptrs.append(a.ctypes.data)
        assert on_dev is None or on_dev == dev, "cubes must all be on the device or all on the host"
        on_dev = dev
    parr = (C.c_void_p * len(ctxs))(*ptrs)
    tarr = (C.c_int64 * len(ctxs))(*[int(t) for t in ts])
    _batch_check(ctxs, lib().lpf_ingest_batch(_ctx_array(ctxs), tarr, parr, int(on_dev or 0), len(ctxs)),
                 "ingest_batch")
    del holders


def detect_batch(ctxs: Sequence["Context"]) -> None:
    _batch_check(ctxs, lib().lpf_detect_batch(_ctx_array(ctxs), len(ctxs)), "detect_batch")


def extract_flux_batch(ctxs: Sequence["Context"]) -> None:
    _batch_check(ctxs, lib().lpf_extract_flux_batch(_ctx_array(ctxs), len(ctxs)), "extract_flux_batch")


LAYER_ORDER = ("conv1.w", "conv1.b", "conv2.w", "conv2.b", "conv3.w", "conv3.b",
               "conv4.w", "conv4.b", "fc1.w", "fc1.b", "fc2.w", "fc2.b")


def pack_weights(wts: dict) -> bytes:
    """Weights dict (PyTorch layouts, float32) -> the blob of lpf_model_create."""
    parts = [np.ascontiguousarray(wts[k], dtype=np.float32).ravel() for k in LAYER_ORDER]
    parts.append(np.array([float(wts.get("alpha", 0.0))], dtype=np.float32))
    blob = np.concatenate(parts).tobytes()
    if len(blob) != lib().lpf_model_weights_bytes():
        raise ValueError("weights have the wrong shapes")
    return blob


class Model:
    def __init__(self, wts: dict, precision: int = PREC_FP32, max_batch: int = 1024,
                 device: str = "cuda:0", stream=None):
        torch = _torch()
        self.blob = pack_weights(wts)
        n = C.c_size_t(0)
        rc = lib().lpf_model_workspace_size(precision, max_batch, C.byref(n))
        if rc != LPF_OK:
            raise LpfError(rc, "model workspace size")
        self.workspace = torch.empty(int(n.value), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        buf = C.create_string_buffer(self.blob, len(self.blob))
        rc = lib().lpf_model_create(buf, len(self.blob), precision, max_batch,
                                    C.c_void_p(self.workspace.data_ptr()), int(n.value),
                                    C.c_void_p(_stream_ptr(stream)), C.byref(h))
        if rc != LPF_OK:
            raise LpfError(rc, "lpf_model_create failed")
        self.h = h
        self.precision = precision
        self.max_batch = max_batch

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.lpf_model_destroy(h)
            self.h = None

    def infer(self, ctxs: List[Context], ids: Optional[Sequence[int]] = None, cap: int = 65536):
        arr = (C.c_void_p * len(ctxs))(*[c.h for c in ctxs])
        mu = np.zeros((cap, 4), dtype=np.float32)
        L = np.zeros((cap, 10), dtype=np.float32)
        src = np.zeros((cap, 2), dtype=np.int32)
        n = C.c_int32(0)
        idp, nid = None, 0
        if ids is not None:
            ida = np.ascontiguousarray(ids, dtype=np.int32)
            idp, nid = C.c_void_p(ida.ctypes.data), len(ida)
        rc = lib().lpf_infer(arr, len(ctxs), self.h, idp, nid, C.c_void_p(mu.ctypes.data),
                             C.c_void_p(L.ctypes.data), C.c_void_p(src.ctypes.data), cap, C.byref(n))
        if rc != LPF_OK:
            raise LpfError(rc, f"infer: {lib().lpf_last_error(ctxs[0].h).decode()}")
        k = n.value
        return mu[:k].copy(), L[:k].copy(), src[:k].copy()

    def infer_async(self, ctxs: List[Context]) -> int:
        """Enqueues inference over the episodes that ended at each context's
        last detect; returns a ticket for collect() (nothing waits)."""
        arr = (C.c_void_p * len(ctxs))(*[c.h for c in ctxs])
        t = C.c_int64(-1)
        rc = lib().lpf_infer_async(arr, len(ctxs), self.h, C.byref(t))
        if rc != LPF_OK:
            raise LpfError(rc, f"infer_async: {lib().lpf_last_error(ctxs[0].h).decode()}")
        return int(t.value)

    def collect(self, ticket: int, cap: Optional[int] = None, strict: bool = True):
        """Waits for a ticket; returns (mu, L, src) as infer() does.  With
        strict=False an overflow of the model's batch is returned, not raised."""
        cap = self.max_batch if cap is None else cap
        mu = np.zeros((cap, 4), dtype=np.float32)
        L = np.zeros((cap, 10), dtype=np.float32)
        src = np.zeros((cap, 2), dtype=np.int32)
        n = C.c_int32(0)
        rc = lib().lpf_infer_collect(self.h, int(ticket), C.c_void_p(mu.ctypes.data), C.c_void_p(L.ctypes.data),
                                     C.c_void_p(src.ctypes.data), cap, C.byref(n))
        if rc != LPF_OK and (strict or rc != LPF_EFULL):
            raise LpfError(rc, "collect")
        k = n.value
        return mu[:k].copy(), L[:k].copy(), src[:k].copy()

    def infer_windows(self, windows, stream=None):
        """windows: torch CUDA float32 [n][16][64] -> (mu [n][4], L [n][10]) torch tensors."""
        torch = _torch()
        assert windows.is_cuda and windows.dtype == torch.float32 and windows.is_contiguous()
        n = windows.shape[0]
        mu = torch.empty((n, 4), dtype=torch.float32, device=windows.device)
        L = torch.empty((n, 10), dtype=torch.float32, device=windows.device)
        rc = lib().lpf_infer_windows(self.h, C.c_void_p(windows.data_ptr()), n, C.c_void_p(mu.data_ptr()),
                                     C.c_void_p(L.data_ptr()), C.c_void_p(_stream_ptr(stream)))
        if rc != LPF_OK:
            raise LpfError(rc, "infer_windows")
        return mu, L

    def infer_windows_static(self, windows, mu, L, stream=None):
        """The allocation-free form: the network's intermediate buffers live in
        the library's static device array; mu [n][4] and L [n][10] are the
        caller's torch CUDA float32 tensors (n <= 32).  Returns the status."""
        torch = _torch()
        assert windows.is_cuda and windows.dtype == torch.float32 and windows.is_contiguous()
        assert mu.is_contiguous() and L.is_contiguous()
        return int(lib().lpf_infer_windows_static(self.h, C.c_void_p(windows.data_ptr()), int(windows.shape[0]),
                                                  C.c_void_p(mu.data_ptr()), C.c_void_p(L.data_ptr()),
                                                  C.c_void_p(_stream_ptr(stream))))


FRAME_DTYPE = np.dtype([("stream_id", "<i4"), ("pad0", "<i4"), ("t", "<i8"), ("arrival_ns", "<i8"),
                        ("done_ns", "<i8"), ("rejected_bands", "<u4"), ("n_peaks", "<i4"),
                        ("n_new", "<i4"), ("n_ended", "<i4"), ("status", "<i4"), ("pad1", "<i4")])


def now_ns() -> int:
    return int(lib().lpf_now_ns())


class Server:
    """Serving loop over several streams (see include/lpf.h).  Frames handed
    to submit() must stay alive until reported done; the server keeps a
    reference to torch tensors until then."""

    def __init__(self, model: "Model", hbm_budget_bytes: int, record: bool = False):
        h = C.c_void_p()
        rc = lib().lpf_server_create(model.h, int(hbm_budget_bytes), 1 if record else 0, C.byref(h))
        if rc != LPF_OK:
            raise LpfError(rc, "lpf_server_create")
        self.h = h
        self.model = model
        self._keep = {}
        self._masks = []
        self._ws = {}       # caller-owned workspaces, released after close
        self._active = {}

    def close_all(self):
        if getattr(self, "h", None) is not None:
            lib().lpf_server_destroy(self.h)
            self.h = None
            self._keep.clear()
            self._ws.clear()

    def __del__(self):
        self.close_all()

    def admit(self, B: int, H: int, W: int, sky_mask=None, grid_rows=None, queue: bool = False,
              own_workspace: bool = True, **params) -> int:
        """Admits a stream; its workspace is a torch uint8 tensor held here
        until close (own_workspace=True), or allocated by the server when the
        stream becomes active.  With queue=True a stream that does not fit the
        budget waits (see is_active) instead of raising LPF_ENOMEM."""
        torch = _torch()
        cfg = default_config(B, H, W, **params)
        keep = []
        if sky_mask is not None:
            m = np.ascontiguousarray(sky_mask, dtype=np.uint8)
            keep.append(m)
            cfg.sky_mask = m.ctypes.data
        if grid_rows is not None:
            r = np.ascontiguousarray(grid_rows, dtype=np.int32)
            keep.append(r)
            cfg.grid_rows = r.ctypes.data
        ws, nbytes = None, 0
        if own_workspace:
            nbytes = workspace_size(cfg)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        sid, act = C.c_int32(-1), C.c_int32(0)
        rc = lib().lpf_server_admit(self.h, C.byref(cfg), C.c_void_p(ws.data_ptr() if ws is not None else None),
                                    nbytes, 1 if queue else 0, C.byref(sid), C.byref(act))
        if rc != LPF_OK:
            raise LpfError(rc, "admit")
        self._ws[int(sid.value)] = ws
        self._active[int(sid.value)] = bool(act.value)
        return int(sid.value)

    def close(self, sid: int):
        rc = lib().lpf_server_close(self.h, int(sid))
        if rc != LPF_OK:
            raise LpfError(rc, "close")
        for key in [k for k in self._keep if k[0] == sid]:
            del self._keep[key]
        self._ws.pop(int(sid), None)
        self._active.pop(int(sid), None)

    def admitted_active(self, sid: int) -> bool:
        """Whether the stream was active when admit() returned."""
        return self._active[int(sid)]

    def submit(self, sid: int, t: int, cube, arrival_ns: Optional[int] = None):
        torch = _torch()
        if isinstance(cube, torch.Tensor):
            assert cube.is_cuda and cube.dtype == torch.float32 and cube.is_contiguous()
            ptr, on_dev = cube.data_ptr(), 1
        else:
            cube = np.ascontiguousarray(cube, dtype=np.float32)
            ptr, on_dev = cube.ctypes.data, 0
        self._keep[(sid, int(t))] = cube
        rc = lib().lpf_server_submit(self.h, int(sid), int(t), C.c_void_p(ptr), on_dev,
                                     int(arrival_ns if arrival_ns is not None else now_ns()))
        if rc != LPF_OK:
            raise LpfError(rc, "submit")

    def poll(self, cap: int = 4096) -> np.ndarray:
        out = np.zeros(cap, dtype=FRAME_DTYPE)
        n = C.c_int32(0)
        rc = lib().lpf_server_poll(self.h, C.c_void_p(out.ctypes.data), cap, C.byref(n))
        if rc != LPF_OK:
            raise LpfError(rc, "poll")
        res = out[:n.value].copy()
        for r in res:
            self._keep.pop((int(r["stream_id"]), int(r["t"])), None)
        return res

    def drain(self):
        rc = lib().lpf_server_drain(self.h)
        if rc != LPF_OK:
            raise LpfError(rc, "drain: frames held by waiting streams")

    def fetch(self, sid: int, t: int, peak_cap: int = 8192, ev_cap: int = 16384, inf_cap: int = 16384):
        peaks = np.zeros(peak_cap, dtype=PEAK_DTYPE)
        ev = np.zeros(ev_cap, dtype=SOURCE_DTYPE)
        mu = np.zeros((inf_cap, 4), dtype=np.float32)
        L = np.zeros((inf_cap, 10), dtype=np.float32)
        ids = np.zeros(inf_cap, dtype=np.int32)
        np_, ne, ni = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        rc = lib().lpf_server_fetch(self.h, int(sid), int(t), C.c_void_p(peaks.ctypes.data), peak_cap,
                                    C.byref(np_), C.c_void_p(ev.ctypes.data), ev_cap, C.byref(ne),
                                    C.c_void_p(mu.ctypes.data), C.c_void_p(L.ctypes.data),
                                    C.c_void_p(ids.ctypes.data), inf_cap, C.byref(ni))
        if rc != LPF_OK:
            raise LpfError(rc, "fetch")
        return (peaks[:np_.value].copy(), ev[:ne.value].copy(), mu[:ni.value].copy(),
                L[:ni.value].copy(), ids[:ni.value].copy())

    def usage(self):
        u, b, n = C.c_size_t(0), C.c_size_t(0), C.c_int32(0)
        lib().lpf_server_usage(self.h, C.byref(u), C.byref(b), C.byref(n))
        return int(u.value), int(b.value), int(n.value)
