"""Python binding of libebof (the C ABI declared in include/ebof.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.  Functions
keep the C names; tensors are checked on the host (device, dtype, contiguity,
size) before their pointers reach a kernel.  There is no fallback: if the
library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libebof.so")

EBOF_OK = 0
EBOF_NO_FLOW = 1
EBOF_E_INVAL = -1
EBOF_E_NOMEM = -2
EBOF_E_AGAIN = -3
EBOF_E_NOTFOUND = -4
EBOF_E_DEVICE = -5
EBOF_E_STATE = -6
EBOF_MASK_FLOW = 1
EBOF_CHAIN_ALWAYS = 2
EBOF_WARM_START = 4
EBOF_VAR_REFINE = 8
EBOF_SURFACE_EXP, EBOF_SURFACE_LINEAR, EBOF_SURFACE_BOUNDED, EBOF_SURFACE_LOG = 0, 1, 2, 3
EBOF_MAX_BATCH = 1024
EBOF_MAX_LEVELS = 8
EBOF_TUNE_OFF = 0
EBOF_TUNE_AUTO = 1
EBOF_TUNE_LEVELS = 8   # lanes-per-patch values per cache line (one per level)
EBOF_TUNE_STAGES = 22  # block counts per cache line (one per internal stage)
EBOF_SIGNAL_SLOTS = 64
EBOF_MAX_OWNED_STREAMS = 16

KERNELS = ["scatter", "denoise_fill", "pack_cols", "edt_cols", "edt_rows", "pyr_down",
           "dis_level", "densify"]


class EbofError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ebof error {code}: {msg}")
        self.code = code


class ebof_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("dt_us", ctypes.c_int64),
        ("n_d", ctypes.c_int32),
        ("n_f", ctypes.c_int32),
        ("alpha", ctypes.c_float),
        ("levels", ctypes.c_int32),
        ("patch", ctypes.c_int32),
        ("stride", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("lambda_reg", ctypes.c_float),
        ("flags", ctypes.c_uint32),
        ("surface", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ebof_window(ctypes.Structure):
    _fields_ = [
        ("params", ctypes.POINTER(ebof_params)),
        ("x", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("t", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("t0_us", ctypes.c_int64),
        ("edge_out", ctypes.c_void_p),
        ("d2_out", ctypes.c_void_p),
        ("pyr_out", ctypes.c_void_p),
        ("pyr_prev", ctypes.c_void_p),
        ("mask", ctypes.c_void_p),
        ("flow_out", ctypes.c_void_p),
        ("n_dropped_dev", ctypes.c_void_p),
        ("flow_init", ctypes.c_void_p),
        ("flow_dense_out", ctypes.c_void_p),
    ]


class ebof_window_events(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("t", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("t0_us", ctypes.c_int64)]


class ebof_ring_slot(ctypes.Structure):
    _fields_ = [("edge", ctypes.c_void_p), ("pyr", ctypes.c_void_p), ("flow", ctypes.c_void_p)]


_lib = None


class ebof_filter_params(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int32), ("gamma", ctypes.c_float * EBOF_MAX_LEVELS),
                ("smooth", ctypes.c_int32 * EBOF_MAX_LEVELS)]


def load():
    """Load libebof.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise RuntimeError(f"{SO_PATH} is missing: build it with paper_2112_10591_amd.build.build()")
    lib = ctypes.CDLL(SO_PATH)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    pp = ctypes.POINTER(ebof_params)
    sig = {
        "ebof_params_default": ([i32, i32, pp], ctypes.c_int),
        "ebof_validate": ([pp], ctypes.c_int),
        "ebof_pyramid_floats": ([pp], i64),
        "ebof_window_scratch_bytes": ([pp], i64),
        "ebof_create": ([ctypes.c_int, P, ctypes.c_size_t, ctypes.POINTER(P)], ctypes.c_int),
        "ebof_destroy": ([P], ctypes.c_int),
        "ebof_last_error": ([P], ctypes.c_char_p),
        "ebof_bin_events": ([P, pp, P, P, P, i64, i64, P, P, P], ctypes.c_int),
        "ebof_edt_surface": ([P, pp, P, P, P, P], ctypes.c_int),
        "ebof_window_surface": ([P, pp, P, P, P, i64, i64, P, P, P, P, P], ctypes.c_int),
        "ebof_flow": ([P, pp, P, P, P, P, P], ctypes.c_int),
        "ebof_flow_noalloc": ([pp, P, P, P, P, P], ctypes.c_int),
        "ebof_flow_errors": ([P, i32, i32, P, P, P, P, P], ctypes.c_int),
        "ebof_window_end": ([P, i32, i32, P, P, i64, i64, i32, i32, P, P], ctypes.c_int),
        "ebof_window_surface_range": ([P, pp, P, P, i64, P, P, P, P, P, P], ctypes.c_int),
        "ebof_fwl": ([P, pp, P, P, P, P, i64, i64, P, P, P], ctypes.c_int),
        "ebof_flow_warm": ([P, pp, P, P, P, P, P, P, P], ctypes.c_int),
        "ebof_run_batch": ([P, ctypes.POINTER(ebof_window), i32, P], ctypes.c_int),
        "ebof_set_tuning": ([P, ctypes.c_int, ctypes.c_char_p], ctypes.c_int),
        "ebof_stream_open": ([P, pp, ctypes.POINTER(i32)], ctypes.c_int),
        "ebof_stream_close": ([P, i32], ctypes.c_int),
        "ebof_submit": ([P, i32, P, P, P, i64, i64, ctypes.c_int, P, P,
                         ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "ebof_poll": ([P, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(i64)], ctypes.c_int),
        "ebof_drain": ([P], ctypes.c_int),
        "ebof_stream_signal": ([P, i32, u32, P], ctypes.c_int),
        "ebof_stream_wait": ([P, i32, u32, P], ctypes.c_int),
        "ebof_signal_read": ([P, i32, ctypes.POINTER(u32)], ctypes.c_int),
        "ebof_stream_create": ([P, ctypes.POINTER(P)], ctypes.c_int),
        "ebof_run_sequence": ([P, pp, ctypes.POINTER(ebof_window_events), i64, i64, ctypes.POINTER(ebof_ring_slot),
                               i32, ctypes.POINTER(P), i32, i32], ctypes.c_int),
        "ebof_timing_enable": ([P, u32], ctypes.c_int),
        "ebof_timing_read": ([P, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
                             ctypes.c_int),
        "ebof_version": ([], ctypes.c_char_p),
        "ebof_filter_params_default": ([i32, i32, ctypes.POINTER(ebof_filter_params)], ctypes.c_int),
        "ebof_filter_state_floats": ([pp, ctypes.POINTER(ebof_filter_params)], i64),
        "ebof_flow_filter": ([P, pp, ctypes.POINTER(ebof_filter_params), P, P, P, P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def exported_symbols():
    return ["ebof_params_default", "ebof_validate", "ebof_pyramid_floats",
            "ebof_window_scratch_bytes", "ebof_create", "ebof_destroy", "ebof_last_error",
            "ebof_bin_events", "ebof_edt_surface", "ebof_window_surface", "ebof_flow", "ebof_flow_warm", "ebof_flow_noalloc", "ebof_flow_errors", "ebof_fwl", "ebof_window_end", "ebof_window_surface_range", "ebof_run_batch", "ebof_set_tuning",
            "ebof_stream_open", "ebof_stream_close", "ebof_submit", "ebof_poll", "ebof_drain",
            "ebof_stream_signal", "ebof_stream_wait", "ebof_signal_read", "ebof_stream_create", "ebof_run_sequence",
            "ebof_timing_enable", "ebof_timing_read", "ebof_version", "ebof_filter_params_default",
            "ebof_filter_state_floats", "ebof_flow_filter"]


# --------------------------------------------------------------------------
# host-only helpers (no device needed)
# --------------------------------------------------------------------------
def ebof_params_default(width, height, **overrides):
    p = ebof_params()
    rc = load().ebof_params_default(int(width), int(height), ctypes.byref(p))
    if rc != EBOF_OK:
        raise EbofError(rc, load().ebof_last_error(None).decode())
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def ebof_validate(p):
    return load().ebof_validate(ctypes.byref(p))


def ebof_pyramid_floats(p):
    n = load().ebof_pyramid_floats(ctypes.byref(p))
    if n < 0:
        raise EbofError(EBOF_E_INVAL, load().ebof_last_error(None).decode())
    return int(n)


def ebof_window_scratch_bytes(p):
    return int(load().ebof_window_scratch_bytes(ctypes.byref(p)))


def level_sizes(p):
    w, h, out = p.width, p.height, []
    for _ in range(p.levels):
        out.append((w, h))
        w, h = (w + 1) // 2, (h + 1) // 2
    return out


# --------------------------------------------------------------------------
# tensor checks
# --------------------------------------------------------------------------
def _dev(t, dtype, numel, name, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(ctx, rc, ok=(EBOF_OK,)):
    if rc not in ok:
        raise EbofError(rc, load().ebof_last_error(ctx).decode())
    return rc


# --------------------------------------------------------------------------
# context and stage calls
# --------------------------------------------------------------------------
class ebof_ctx:
    """Owns the arena tensor and the library context."""

    def __init__(self, arena_bytes=1 << 30, device=0):
        self.lib = load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        h = ctypes.c_void_p()
        rc = self.lib.ebof_create(int(device), ctypes.c_void_p(self.arena.data_ptr()),
                                  self.arena.numel(), ctypes.byref(h))
        if rc != EBOF_OK:
            raise EbofError(rc, self.lib.ebof_last_error(None).decode())
        self.handle = h
        self._keep = []

    def close(self):
        if self.handle is not None:
            self.lib.ebof_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ebof_create(arena_bytes=1 << 30, device=0):
    return ebof_ctx(arena_bytes, device)


def ebof_destroy(ctx):
    ctx.close()


def ebof_last_error(ctx):
    return load().ebof_last_error(ctx.handle).decode()


def ebof_bin_events(ctx, p, x, y, t, t0_us, edge_out, n_dropped=None, stream=None):
    n = int(x.numel())
    px = _dev(x, torch.uint16, n, "x")
    py = _dev(y, torch.uint16, n, "y")
    pt = _dev(t, torch.int64, n, "t")
    pe = _dev(edge_out, torch.uint8, p.width * p.height, "edge_out")
    pd = _dev(n_dropped, torch.uint64, 1, "n_dropped", optional=True)
    return _check(ctx.handle, ctx.lib.ebof_bin_events(ctx.handle, ctypes.byref(p), px, py, pt, n,
                                                      int(t0_us), pe, pd, _stream(stream)))


def ebof_edt_surface(ctx, p, edge, pyr_out, d2_out=None, stream=None):
    N = p.width * p.height
    pe = _dev(edge, torch.uint8, N, "edge")
    pp = _dev(pyr_out, torch.float32, ebof_pyramid_floats(p), "pyr_out")
    pd = _dev(d2_out, torch.int32, N, "d2_out", optional=True)
    return _check(ctx.handle, ctx.lib.ebof_edt_surface(ctx.handle, ctypes.byref(p), pe, pd, pp,
                                                       _stream(stream)))


def ebof_window_surface(ctx, p, x, y, t, t0_us, edge_out, pyr_out, d2_out=None, n_dropped=None, stream=None):
    n = int(x.numel())
    N = p.width * p.height
    px = _dev(x, torch.uint16, n, "x")
    py = _dev(y, torch.uint16, n, "y")
    pt = _dev(t, torch.int64, n, "t")
    pe = _dev(edge_out, torch.uint8, N, "edge_out")
    pn = _dev(n_dropped, torch.uint64, 1, "n_dropped", optional=True)
    pd = _dev(d2_out, torch.int32, N, "d2_out", optional=True)
    pp = _dev(pyr_out, torch.float32, ebof_pyramid_floats(p), "pyr_out")
    return _check(ctx.handle, ctx.lib.ebof_window_surface(ctx.handle, ctypes.byref(p), px, py, pt, n, int(t0_us),
                                                          pe, pn, pd, pp, _stream(stream)))


def ebof_flow(ctx, p, pyr_prev, pyr_curr, flow_out, mask=None, stream=None):
    P = ebof_pyramid_floats(p)
    N = p.width * p.height
    a = _dev(pyr_prev, torch.float32, P, "pyr_prev")
    b = _dev(pyr_curr, torch.float32, P, "pyr_curr")
    m = _dev(mask, torch.uint8, N, "mask", optional=True)
    f = _dev(flow_out, torch.float32, 2 * N, "flow_out")
    return _check(ctx.handle, ctx.lib.ebof_flow(ctx.handle, ctypes.byref(p), a, b, m, f,
                                                _stream(stream)))


def ebof_flow_warm(ctx, p, pyr_prev, pyr_curr, flow_out, flow_init=None, flow_dense_out=None, mask=None,
                   stream=None):
    """ebof_flow with the coarsest level started from flow_init (the previous
    pair's flow before masking); flow_dense_out receives this flow before
    masking."""
    P = ebof_pyramid_floats(p)
    N = p.width * p.height
    a = _dev(pyr_prev, torch.float32, P, "pyr_prev")
    b = _dev(pyr_curr, torch.float32, P, "pyr_curr")
    m = _dev(mask, torch.uint8, N, "mask", optional=True)
    fi = _dev(flow_init, torch.float32, 2 * N, "flow_init", optional=True)
    f = _dev(flow_out, torch.float32, 2 * N, "flow_out")
    fd = _dev(flow_dense_out, torch.float32, 2 * N, "flow_dense_out", optional=True)
    return _check(ctx.handle, ctx.lib.ebof_flow_warm(ctx.handle, ctypes.byref(p), a, b, m, fi, f, fd,
                                                     _stream(stream)))


def ebof_filter_params_default(width, height, **overrides):
    """Sec. IV-A's filter settings for a width x height sensor; overrides:
    layers=, gamma=[...], smooth=[...] (finest layer first)."""
    fp = ebof_filter_params()
    rc = load().ebof_filter_params_default(int(width), int(height), ctypes.byref(fp))
    if rc != EBOF_OK:
        raise EbofError(rc, load().ebof_last_error(None).decode())
    if "layers" in overrides:
        fp.layers = int(overrides["layers"])
    for name in ("gamma", "smooth"):
        if name in overrides:
            arr = getattr(fp, name)
            for l, v in enumerate(overrides[name]):
                arr[l] = v
    return fp


def ebof_filter_state_floats(p, fp):
    n = load().ebof_filter_state_floats(ctypes.byref(p), ctypes.byref(fp))
    if n < 0:
        raise EbofError(EBOF_E_INVAL, load().ebof_last_error(None).decode())
    return int(n)


def ebof_flow_filter(ctx, p, fp, pyr_prev, pyr_curr, state, flow_out, mask=None, stream=None):
    """One step of the update-prediction flow filter (state in/out)."""
    P = ebof_pyramid_floats(p)
    N = p.width * p.height
    a = _dev(pyr_prev, torch.float32, P, "pyr_prev")
    b = _dev(pyr_curr, torch.float32, P, "pyr_curr")
    m = _dev(mask, torch.uint8, N, "mask", optional=True)
    s = _dev(state, torch.float32, ebof_filter_state_floats(p, fp), "state")
    f = _dev(flow_out, torch.float32, 2 * N, "flow_out")
    return _check(ctx.handle, ctx.lib.ebof_flow_filter(ctx.handle, ctypes.byref(p), ctypes.byref(fp), a, b, m, s,
                                                       f, _stream(stream)))


def ebof_flow_noalloc(p, pyr_prev, pyr_curr, flow_out, mask=None, stream=None):
    """ebof_flow without a context, on the current device (scratch in a
    fixed device array: nothing is allocated)."""
    P = ebof_pyramid_floats(p)
    N = p.width * p.height
    a = _dev(pyr_prev, torch.float32, P, "pyr_prev")
    b = _dev(pyr_curr, torch.float32, P, "pyr_curr")
    m = _dev(mask, torch.uint8, N, "mask", optional=True)
    f = _dev(flow_out, torch.float32, 2 * N, "flow_out")
    return _check(None, load().ebof_flow_noalloc(ctypes.byref(p), a, b, m, f, _stream(stream)))


def ebof_window_end(ctx, width, height, x, y, i0, area, k_events, range_out=None, stream=None):
    """End of the adaptive window from event i0 (area event count rule).
    With range_out (a device int64[2] tensor) the call is asynchronous and
    fills it; without, returns (i0, end) after waiting for the stream."""
    n = int(x.numel())
    a = _dev(x, torch.uint16, n, "x")
    b = _dev(y, torch.uint16, n, "y")
    out = range_out if range_out is not None else torch.empty(2, dtype=torch.int64, device=x.device)
    r = _dev(out, torch.int64, 2, "range_out")
    _check(ctx.handle, ctx.lib.ebof_window_end(ctx.handle, int(width), int(height), a, b, n, int(i0), int(area),
                                               int(k_events), r, _stream(stream)))
    if range_out is not None:
        return None
    _sync(stream)
    return tuple(int(v) for v in out.cpu().tolist())


def ebof_window_surface_range(ctx, p, x, y, range_dev, edge_out, pyr_out, d2_out=None, n_dropped=None, stream=None):
    """ebof_window_surface of the events in the device index range range_dev."""
    n = int(x.numel())
    N = p.width * p.height
    a = _dev(x, torch.uint16, n, "x")
    b = _dev(y, torch.uint16, n, "y")
    r = _dev(range_dev, torch.int64, 2, "range_dev")
    e = _dev(edge_out, torch.uint8, N, "edge_out")
    pr = _dev(pyr_out, torch.float32, ebof_pyramid_floats(p), "pyr_out")
    d2 = _dev(d2_out, torch.int32, N, "d2_out", optional=True)
    nd = _dev(n_dropped, torch.uint64, 1, "n_dropped", optional=True)
    return _check(ctx.handle, ctx.lib.ebof_window_surface_range(ctx.handle, ctypes.byref(p), a, b, n, r, e, nd, d2,
                                                                pr, _stream(stream)))


def _sync(stream):
    (stream if stream is not None else torch.cuda.current_stream()).synchronize()


def ebof_flow_errors(ctx, width, height, flow, gt, mask=None, stream=None):
    """(AEE, outlier fraction, pixels counted) of flow against gt over mask
    (Sec. IV); waits for the stream."""
    N = int(width) * int(height)
    f = _dev(flow, torch.float32, 2 * N, "flow")
    g = _dev(gt, torch.float32, 2 * N, "gt")
    m = _dev(mask, torch.uint8, N, "mask", optional=True)
    out = torch.empty(3, dtype=torch.float64, device=flow.device)
    _check(ctx.handle, ctx.lib.ebof_flow_errors(ctx.handle, int(width), int(height), f, g, m,
                                                ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    _sync(stream)
    a, o, n = out.cpu().tolist()
    return a, o, int(n)


def ebof_fwl(ctx, p, x, y, t, t0_us, flow, pol=None, stream=None):
    """(FWL, variance compensated, variance uncompensated) of the window's
    events under flow (Sec. IV); waits for the stream."""
    ne = int(x.numel())
    N = p.width * p.height
    a = _dev(x, torch.uint16, ne, "x")
    b = _dev(y, torch.uint16, ne, "y")
    c = _dev(t, torch.int64, ne, "t")
    q = _dev(pol, torch.int8, ne, "pol", optional=True)
    f = _dev(flow, torch.float32, 2 * N, "flow")
    out = torch.empty(3, dtype=torch.float64, device=flow.device)
    _check(ctx.handle, ctx.lib.ebof_fwl(ctx.handle, ctypes.byref(p), a, b, c, q, ne, int(t0_us), f,
                                        ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    _sync(stream)
    return tuple(out.cpu().tolist())


def ebof_set_tuning(ctx, mode=EBOF_TUNE_AUTO, cache_path=None):
    """Launch-shape tuning of the batched form (EBOF_TUNE_AUTO / EBOF_TUNE_OFF),
    optionally with a cache file of tuned layouts."""
    path = None if cache_path is None else os.fsencode(cache_path)
    return _check(ctx.handle, ctx.lib.ebof_set_tuning(ctx.handle, int(mode), path))


def batch_layout_key(windows):
    """The layout string of a batch as the tuning cache file names it."""
    out = []
    for w in windows:
        p = w["params"]
        flow = 1 if w.get("pyr_prev") is not None else 0
        out.append(f"{p.width},{p.height},{p.levels},{p.stride},{flow},0;")
    return "".join(out)


def ebof_run_batch(ctx, windows, stream=None):
    """windows: list of dicts with keys params, x, y, t, t0_us, edge_out, pyr_out and
    optionally d2_out, pyr_prev, mask, flow_out, n_dropped, flow_init, flow_dense_out."""
    n = len(windows)
    if not 1 <= n <= EBOF_MAX_BATCH:
        raise ValueError("batch size out of range")
    arr = (ebof_window * n)()
    keep = []
    for i, w in enumerate(windows):
        p = w["params"]
        keep.append(p)
        N = p.width * p.height
        P = ebof_pyramid_floats(p)
        ne = int(w["x"].numel())
        a = arr[i]
        a.params = ctypes.pointer(p)
        a.x = _dev(w["x"], torch.uint16, ne, "x")
        a.y = _dev(w["y"], torch.uint16, ne, "y")
        a.t = _dev(w["t"], torch.int64, ne, "t")
        a.n = ne
        a.t0_us = int(w["t0_us"])
        a.edge_out = _dev(w["edge_out"], torch.uint8, N, "edge_out")
        a.d2_out = _dev(w.get("d2_out"), torch.int32, N, "d2_out", optional=True)
        a.pyr_out = _dev(w["pyr_out"], torch.float32, P, "pyr_out")
        a.pyr_prev = _dev(w.get("pyr_prev"), torch.float32, P, "pyr_prev", optional=True)
        a.mask = _dev(w.get("mask"), torch.uint8, N, "mask", optional=True)
        need_flow = w.get("pyr_prev") is not None
        a.flow_out = _dev(w.get("flow_out"), torch.float32, 2 * N, "flow_out", optional=not need_flow)
        a.n_dropped_dev = _dev(w.get("n_dropped"), torch.uint64, 1, "n_dropped", optional=True)
        a.flow_init = _dev(w.get("flow_init"), torch.float32, 2 * N, "flow_init", optional=True)
        a.flow_dense_out = _dev(w.get("flow_dense_out"), torch.float32, 2 * N, "flow_dense_out", optional=True)
    return _check(ctx.handle, ctx.lib.ebof_run_batch(ctx.handle, arr, n, _stream(stream)))


# --------------------------------------------------------------------------
# cross-stream ordering
# --------------------------------------------------------------------------
def ebof_stream_signal(ctx, slot, value, stream=None):
    return _check(ctx.handle, ctx.lib.ebof_stream_signal(ctx.handle, int(slot), int(value) & 0xFFFFFFFF,
                                                         _stream(stream)))


def ebof_stream_wait(ctx, slot, value, stream=None):
    return _check(ctx.handle, ctx.lib.ebof_stream_wait(ctx.handle, int(slot), int(value) & 0xFFFFFFFF,
                                                       _stream(stream)))


def ebof_signal_read(ctx, slot):
    v = ctypes.c_uint32()
    _check(ctx.handle, ctx.lib.ebof_signal_read(ctx.handle, int(slot), ctypes.byref(v)))
    return v.value


def ebof_stream_create(ctx):
    """A context-owned HIP stream on a hardware queue of its own, wrapped as a
    torch stream (valid until the context is closed)."""
    s = ctypes.c_void_p()
    _check(ctx.handle, ctx.lib.ebof_stream_create(ctx.handle, ctypes.byref(s)))
    return torch.cuda.ExternalStream(s.value)


class Sequence:
    """Arguments of ebof_run_sequence built once (device pointers of every
    window's events, the ring slots, the streams), so that a call issues a
    whole run of windows with one crossing into the library.
    windows: dicts with x, y, t (device tensors) and t0 (window i of the
    list is window k_lo + i of a run); ring: dicts with edge (uint8, W*H),
    pyr (float32, pyramid floats) and flow (float32, 2*W*H); streams: torch
    streams (e.g. from ebof_stream_create)."""

    def __init__(self, ctx, p, windows, ring, streams, slot0=0):
        self.ctx, self.p, self.slot0 = ctx, p, int(slot0)
        N = p.width * p.height
        P = ebof_pyramid_floats(p)
        self.win = (ebof_window_events * max(1, len(windows)))()
        for i, w in enumerate(windows):
            n = int(w["x"].numel())
            self.win[i] = ebof_window_events(_dev(w["x"], torch.uint16, n, "x"), _dev(w["y"], torch.uint16, n, "y"),
                                             _dev(w["t"], torch.int64, n, "t"), n, int(w["t0"]))
        self.ring = (ebof_ring_slot * len(ring))()
        for i, r in enumerate(ring):
            self.ring[i] = ebof_ring_slot(_dev(r["edge"], torch.uint8, N, "edge"), _dev(r["pyr"], torch.float32, P, "pyr"),
                                          _dev(r["flow"], torch.float32, 2 * N, "flow"))
        self.streams = (ctypes.c_void_p * len(streams))(*[s.cuda_stream for s in streams])
        self.n_win, self.n_ring, self.n_streams = len(windows), len(ring), len(streams)

    def run(self, k_lo, k_hi):
        """Issues windows k_lo .. k_hi-1 (the events of window k_lo + i are
        windows[i])."""
        if k_hi - k_lo > self.n_win:
            raise ValueError("more windows than the sequence holds")
        lib = self.ctx.lib
        _check(self.ctx.handle, lib.ebof_run_sequence(self.ctx.handle, ctypes.byref(self.p), self.win, int(k_lo),
                                                      int(k_hi), self.ring, self.n_ring, self.streams, self.n_streams,
                                                      self.slot0))


EBOF_TIMING_SPAN = 0x80000000


def ebof_timing_enable(ctx, kernels, span=False):
    """Time every launch of the named kernels (span: one event pair around
    the launches of one kernel that a call makes back to back)."""
    mask = EBOF_TIMING_SPAN if span else 0
    for k in kernels:
        mask |= 1 << KERNELS.index(k)
    return _check(ctx.handle, ctx.lib.ebof_timing_enable(ctx.handle, mask))


def ebof_timing_read(ctx, kernel):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(ctx.handle, ctx.lib.ebof_timing_read(ctx.handle, KERNELS.index(kernel), ctypes.byref(ms),
                                                ctypes.byref(cnt)))
    return ms.value, cnt.value


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------
def ebof_stream_open(ctx, p):
    sid = ctypes.c_int32()
    _check(ctx.handle, ctx.lib.ebof_stream_open(ctx.handle, ctypes.byref(p), ctypes.byref(sid)))
    ctx._keep.append(p)
    return sid.value


def ebof_stream_close(ctx, sid):
    return _check(ctx.handle, ctx.lib.ebof_stream_close(ctx.handle, int(sid)))


def ebof_submit(ctx, sid, p, x, y, t, t0_us, flow_out, mask_out):
    """Host (numpy) or device (tensor) events; device outputs.  Returns the
    ticket, or None when the queue is full (EBOF_E_AGAIN)."""
    import numpy as np
    N = p.width * p.height
    f = _dev(flow_out, torch.float32, 2 * N, "flow_out")
    m = _dev(mask_out, torch.uint8, N, "mask_out")
    ticket = ctypes.c_uint64()
    if isinstance(x, torch.Tensor):
        n = int(x.numel())
        args = (_dev(x, torch.uint16, n, "x"), _dev(y, torch.uint16, n, "y"),
                _dev(t, torch.int64, n, "t"), n, int(t0_us), 1)
    else:
        x = np.ascontiguousarray(x, np.uint16)
        y = np.ascontiguousarray(y, np.uint16)
        t = np.ascontiguousarray(t, np.int64)
        n = len(x)
        if len(y) != n or len(t) != n:
            raise ValueError("x, y, t lengths differ")
        args = (ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(y.ctypes.data),
                ctypes.c_void_p(t.ctypes.data), n, int(t0_us), 0)
    rc = ctx.lib.ebof_submit(ctx.handle, int(sid), *args, f, m, ctypes.byref(ticket))
    if rc == EBOF_E_AGAIN:
        return None
    _check(ctx.handle, rc)
    return ticket.value


def ebof_poll(ctx, ticket, with_latency=False):
    """Returns None while pending, else the window status (EBOF_OK /
    EBOF_NO_FLOW), or (status, latency in seconds) with with_latency."""
    st = ctypes.c_int32()
    lat = ctypes.c_int64()
    rc = ctx.lib.ebof_poll(ctx.handle, ctypes.c_uint64(ticket), ctypes.byref(st), ctypes.byref(lat))
    if rc == EBOF_E_AGAIN:
        return None
    _check(ctx.handle, rc)
    return (st.value, lat.value * 1e-9) if with_latency else st.value


def ebof_drain(ctx):
    return _check(ctx.handle, ctx.lib.ebof_drain(ctx.handle))
