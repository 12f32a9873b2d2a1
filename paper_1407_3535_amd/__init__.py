"""Python binding of libzts (exhaustive ZNCC template search on MI355X).

A thin ctypes layer over the C ABI declared in ``include/zts.h``: the
functions below carry the same names and only marshal arguments (numpy
arrays and torch tensors to pointers, structs to dicts).  Every step of a
search runs in the library's HIP kernels; there is no fallback.  The library
must have been built (``python -m paper_1407_3535_amd.build`` or
``__graft_entry__.build()``); loading fails loudly otherwise.

torch is imported first so that the library binds to the HIP runtime torch
already loaded (one runtime per process); torch provides device memory and
streams for the ``*_device`` entry points.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:  # one HIP runtime per process: torch's, when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzts.so")

ZTS_FULL, ZTS_FULL_MFMA, ZTS_TE_FIXED, ZTS_EGS, ZTS_OPTA, ZTS_OPTA_PAPER = 0, 1, 2, 3, 4, 5
MODES = {"full": ZTS_FULL, "full_mfma": ZTS_FULL_MFMA, "te_fixed": ZTS_TE_FIXED, "egs": ZTS_EGS, "opta": ZTS_OPTA,
         "opta_paper": ZTS_OPTA_PAPER}

STATUS = {0: "ok", -1: "invalid argument", -2: "size", -3: "degenerate template", -4: "unknown image",
          -5: "HBM budget exhausted", -6: "not ready", -7: "busy", -8: "timed out", -9: "cancelled",
          -10: "device error", -11: "out of memory", -12: "not prepared"}

EXPORTS = ["zts_params_default", "zts_params_check", "zts_create", "zts_destroy", "zts_status_str", "zts_image_load",
           "zts_image_load_device", "zts_image_unload", "zts_prepare", "zts_prep_query", "zts_prep_image",
           "zts_search", "zts_search_device", "zts_search_device_noalloc", "zts_search_batch", "zts_search_batch_pruned", "zts_search_batch_pruned_device", "zts_tune_batch", "zts_submit", "zts_submit_batch", "zts_poll",
           "zts_wait", "zts_cancel", "zts_pending", "zts_debug_full_map", "zts_debug_autocorr", "zts_debug_blur"]


class ZtsError(RuntimeError):
    def __init__(self, code, where=""):
        super().__init__(f"{where}: zts status {code} ({STATUS.get(code, '?')})")
        self.code = code


class CtxParams(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget_bytes", C.c_uint64), ("max_inflight", C.c_int32),
                ("max_queued", C.c_int32), ("tune_cache", C.c_char_p)]


class TuneEntry(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("single_ms", C.c_float), ("shared_ms", C.c_float),
                ("multi_min", C.c_int32), ("pad", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("rho_th", C.c_double), ("rho_max", C.c_double), ("margin", C.c_double), ("xi", C.c_double),
                ("group_h", C.c_int32), ("group_w", C.c_int32), ("h0", C.c_int32), ("w0", C.c_int32),
                ("dh", C.c_int32), ("dw", C.c_int32), ("h_max", C.c_int32), ("blur_kind", C.c_int32),
                ("sigma_step", C.c_double), ("sigma_max", C.c_double), ("max_iters", C.c_int32),
                ("refine_radius", C.c_int32), ("timing", C.c_int32), ("egs_estimate", C.c_int32),
                ("rho_tc", C.c_double), ("egs_shape", C.c_int32), ("pad0", C.c_int32), ("accept_xi", C.c_double),
                ("rho_floor", C.c_double), ("floor_prune", C.c_int32), ("pad1", C.c_int32),
                ("tile_dense_min", C.c_int32), ("pad2", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("y", C.c_int32), ("x", C.c_int32), ("rho", C.c_double), ("rho32", C.c_float),
                ("pad0", C.c_int32), ("num", C.c_int64), ("den_t", C.c_int64), ("den_r", C.c_int64),
                ("n_locations", C.c_int64), ("n_centres", C.c_int64), ("n_eliminated", C.c_int64),
                ("n_survivors", C.c_int64), ("n_computed", C.c_int64), ("group_h", C.c_int32),
                ("group_w", C.c_int32), ("best0", C.c_double), ("best0_y", C.c_int32), ("best0_x", C.c_int32),
                ("device_ms", C.c_float), ("status", C.c_int32), ("phase_ms", C.c_float * 6),
                ("latency_ms", C.c_float), ("queue_ms", C.c_float), ("batch_size", C.c_int32),
                ("above_floor", C.c_int32), ("n_dense", C.c_int64), ("n_sparse", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k in Result._names}
        d["phase_ms"] = list(self.phase_ms)
        return d


Result._names = [k for k, _ in Result._fields_ if not k.startswith("pad") and k != "phase_ms"]


def _current_stream(device=None) -> int:
    """Handle of torch's current HIP stream on `device` (the current device when None)."""
    if device is None:
        device = torch.cuda.current_device()
    return torch._C._cuda_getCurrentRawStream(device)


class EgsStep(C.Structure):
    _fields_ = [("h", C.c_int32), ("w", C.c_int32), ("cc", C.c_int64), ("cr", C.c_int64), ("ct", C.c_int64),
                ("accepted", C.c_int32), ("pad0", C.c_int32)]


class OptaStep(C.Structure):
    _fields_ = [("k", C.c_int32), ("d", C.c_int32), ("passes", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
                ("accepted", C.c_int32), ("sigma", C.c_double), ("reverted", C.c_int64), ("cost", C.c_int64)]


class PrepInfo(C.Structure):
    _fields_ = [("mode", C.c_int32), ("m", C.c_int32), ("n", C.c_int32), ("group_h", C.c_int32),
                ("group_w", C.c_int32), ("radius", C.c_int32), ("cost", C.c_int64), ("n_egs", C.c_int32),
                ("n_opta", C.c_int32), ("egs", EgsStep * 64), ("opta", OptaStep * 16), ("prepare_ms", C.c_float),
                ("pad0", C.c_int32)]

    def as_dict(self):
        egs = [dict(h=s.h, w=s.w, cc=s.cc, cr=s.cr, ct=s.ct, accepted=bool(s.accepted))
               for s in self.egs[:self.n_egs]]
        opta = [dict(k=s.k, d=s.d, sigma=s.sigma, passes=s.passes, reverted=s.reverted, h=s.h, w=s.w,
                     cost=s.cost, accepted=bool(s.accepted)) for s in self.opta[:self.n_opta]]
        return dict(mode=self.mode, m=self.m, n=self.n, h=self.group_h, w=self.group_w, radius=self.radius,
                    cost=self.cost, egs=egs, opta=opta, prepare_ms=self.prepare_ms)


_lib = None


def lib():
    """Loads libzts.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1407_3535_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.zts_params_default.argtypes = [C.POINTER(Params)]
        L.zts_params_default.restype = None
        L.zts_params_check.argtypes = [C.POINTER(Params)]
        L.zts_create.argtypes = [C.POINTER(CtxParams), C.POINTER(vp)]
        L.zts_destroy.argtypes = [vp]
        L.zts_destroy.restype = None
        L.zts_status_str.argtypes = [i32]
        L.zts_status_str.restype = C.c_char_p
        L.zts_image_load.argtypes = [vp, vp, i32, i32, i64, C.POINTER(i32)]
        L.zts_image_load_device.argtypes = [vp, vp, i32, i32, i64, vp, C.POINTER(i32)]
        L.zts_image_unload.argtypes = [vp, i32]
        L.zts_prepare.argtypes = [vp, i32, i32, i32, i32, C.POINTER(Params), vp]
        L.zts_prep_query.argtypes = [vp, i32, i32, i32, i32, C.POINTER(PrepInfo)]
        L.zts_prep_image.argtypes = [vp, i32, i32, i32, i32, vp]
        L.zts_search.argtypes = [vp, i32, vp, i32, i32, i64, i32, C.POINTER(Params), C.POINTER(Result), vp]
        L.zts_search_device.argtypes = [vp, i32, vp, i32, i32, i64, i32, C.POINTER(Params), vp,
                                        C.POINTER(Result)]
        L.zts_search_device_noalloc.argtypes = L.zts_search_device.argtypes
        L.zts_search_batch.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
        L.zts_search_batch_pruned.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, C.POINTER(Params), vp]
        L.zts_search_batch_pruned_device.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, C.POINTER(Params), vp, vp]
        L.zts_tune_batch.argtypes = [vp, i32, i32, vp, vp, vp]
        L.zts_submit.argtypes = [vp, i32, vp, i32, i32, i64, i32, C.POINTER(Params), C.POINTER(C.c_uint64)]
        L.zts_submit_batch.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, C.POINTER(Params), C.POINTER(C.c_uint64)]
        L.zts_poll.argtypes = [vp, C.c_uint64, C.POINTER(Result)]
        L.zts_wait.argtypes = [vp, C.c_uint64, i64, C.POINTER(Result)]
        L.zts_cancel.argtypes = [vp, C.c_uint64]
        L.zts_pending.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.zts_debug_full_map.argtypes = [vp, i32, vp, i32, i32, i64, vp, vp, vp]
        L.zts_debug_autocorr.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp, vp]
        L.zts_debug_blur.argtypes = [vp, vp, i32, i32, vp, i32, vp]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is C.c_int:
                f.restype = i32
        _lib = L
    return _lib


def _check(rc, where):
    if rc != 0:
        raise ZtsError(rc, where)


def _u8(a):
    a = np.asarray(a)
    if a.dtype != np.uint8 or a.ndim != 2 or a.strides[1] != 1:
        a = np.ascontiguousarray(a, dtype=np.uint8)
    return a


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def zts_params_default(**overrides) -> Params:
    p = Params()
    lib().zts_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def zts_params_check(params: Params) -> int:
    """ZTS_OK (0) when every field is in range, else ZTS_E_ARG (-1); host only."""
    return lib().zts_params_check(C.byref(params))


def zts_status_str(code: int) -> str:
    return lib().zts_status_str(code).decode()


def zts_create(device: int = 0, hbm_budget_bytes: int = 0, max_inflight: int = 0, max_queued: int = 0,
               tune_cache: str | None = None):
    h = C.c_void_p()
    cache = tune_cache.encode() if tune_cache else None
    _check(lib().zts_create(C.byref(CtxParams(device, hbm_budget_bytes, max_inflight, max_queued, cache)),
                            C.byref(h)), "zts_create")
    return h


def zts_tune_batch(ctx, image: int, sizes) -> list:
    """Times the two batched MFMA kernels for each (m, n) and keeps the routes in the context."""
    sizes = [(int(m), int(n)) for m, n in sizes]
    k = len(sizes)
    ms = (C.c_int32 * k)(*[s[0] for s in sizes])
    ns = (C.c_int32 * k)(*[s[1] for s in sizes])
    out = (TuneEntry * k)()
    _check(lib().zts_tune_batch(ctx, image, k, ms, ns, out), "zts_tune_batch")
    return [{"m": e.m, "n": e.n, "single_ms": e.single_ms, "shared_ms": e.shared_ms, "multi_min": e.multi_min}
            for e in out]


def zts_destroy(ctx) -> None:
    lib().zts_destroy(ctx)


def zts_image_load(ctx, img) -> int:
    img = _u8(img)
    i = C.c_int32()
    _check(lib().zts_image_load(ctx, img.ctypes.data, img.shape[0], img.shape[1], img.strides[0], C.byref(i)),
           "zts_image_load")
    return i.value


def zts_image_load_device(ctx, tensor, stream=None) -> int:
    """tensor: a 2-D uint8 torch tensor on the GPU (rows may be strided)."""
    rows, cols = tensor.shape
    s = stream if stream is not None else _current_stream(tensor.device.index)
    i = C.c_int32()
    _check(lib().zts_image_load_device(ctx, tensor.data_ptr(), rows, cols, tensor.stride(0), s, C.byref(i)),
           "zts_image_load_device")
    return i.value


def zts_image_unload(ctx, image: int) -> None:
    _check(lib().zts_image_unload(ctx, image), "zts_image_unload")


def zts_prepare(ctx, image: int, m: int, n: int, mode, params: Params | None = None) -> None:
    p = params if params is not None else zts_params_default()
    _check(lib().zts_prepare(ctx, image, m, n, _mode(mode), C.byref(p), None), "zts_prepare")


def zts_prep_query(ctx, image: int, m: int, n: int, mode) -> dict:
    info = PrepInfo()
    _check(lib().zts_prep_query(ctx, image, m, n, _mode(mode), C.byref(info)), "zts_prep_query")
    return info.as_dict()


def zts_prep_image(ctx, image: int, m: int, n: int, shape, mode="opta") -> np.ndarray:
    out = np.zeros(shape, np.uint8)
    _check(lib().zts_prep_image(ctx, image, m, n, _mode(mode), out.ctypes.data), "zts_prep_image")
    return out


def zts_search(ctx, image: int, tpl, mode, params: Params | None = None) -> dict:
    tpl = _u8(tpl)
    p = params if params is not None else zts_params_default()
    r = Result()
    rc = lib().zts_search(ctx, image, tpl.ctypes.data, tpl.shape[0], tpl.shape[1], tpl.strides[0], _mode(mode),
                          C.byref(p), C.byref(r), None)
    _check(rc, "zts_search")
    return r.as_dict()


def zts_search_decision(ctx, image: int, image_shape, tpl, mode, params: Params | None = None):
    """zts_search with the per-location decision map (1 centre, 3 window, 2 survivor, 0 eliminated)."""
    tpl = _u8(tpl)
    p = params if params is not None else zts_params_default()
    r = Result()
    Ly, Lx = image_shape[0] - tpl.shape[0] + 1, image_shape[1] - tpl.shape[1] + 1
    if Ly < 1 or Lx < 1:
        raise ZtsError(-2, "zts_search")
    dec = np.full((Ly, Lx), -1, np.int8)
    rc = lib().zts_search(ctx, image, tpl.ctypes.data, tpl.shape[0], tpl.shape[1], tpl.strides[0], _mode(mode),
                          C.byref(p), C.byref(r), dec.ctypes.data)
    _check(rc, "zts_search")
    return r.as_dict(), dec


def zts_search_device(ctx, image: int, tpl_tensor, mode, params: Params | None = None, stream=None,
                      out: Result | None = None):
    """One search of a device template (read in place after the caller's stream).  Returns a dict, or, with
    `out`, fills that Result and returns it (no per-call allocation: for loops that search repeatedly)."""
    p = params if params is not None else zts_params_default()
    s = stream if stream is not None else _current_stream(tpl_tensor.device.index)
    r = out if out is not None else Result()
    m, n = tpl_tensor.shape
    _check(lib().zts_search_device(ctx, image, tpl_tensor.data_ptr(), m, n, tpl_tensor.stride(0), _mode(mode),
                                   C.byref(p), s, C.byref(r)), "zts_search_device")
    return r if out is not None else r.as_dict()


def zts_search_device_noalloc(ctx, image: int, tpl_tensor, mode, params: Params | None = None, stream=None,
                              out: Result | None = None):
    """zts_search_device with the query's scratch in the library's static device array (allocates nothing;
    the image's statistics and the mode's tables must be resident already)."""
    p = params if params is not None else zts_params_default()
    s = stream if stream is not None else _current_stream(tpl_tensor.device.index)
    r = out if out is not None else Result()
    m, n = tpl_tensor.shape
    _check(lib().zts_search_device_noalloc(ctx, image, tpl_tensor.data_ptr(), m, n, tpl_tensor.stride(0),
                                           _mode(mode), C.byref(p), s, C.byref(r)), "zts_search_device_noalloc")
    return r if out is not None else r.as_dict()


def zts_search_batch(ctx, image: int, tpls) -> list:
    """Exhaustive search of many host templates in one call (int8 MFMA); one dict per template."""
    tpls, ptrs, ms, ns, st = _tpl_arrays(tpls)
    k = len(tpls)
    out = (Result * k)()
    _check(lib().zts_search_batch(ctx, image, k, ptrs, ms, ns, st, out), "zts_search_batch")
    return [r.as_dict() for r in out]


def zts_search_batch_pruned(ctx, image: int, tpls, mode, params: Params | None = None) -> list:
    """Transitive-elimination search of many host templates in one call (scan 1 shared by the templates of
    one size); one dict per template, each equal to zts_search's."""
    tpls, ptrs, ms, ns, st = _tpl_arrays(tpls)
    k = len(tpls)
    out = (Result * k)()
    p = params if params is not None else zts_params_default()
    _check(lib().zts_search_batch_pruned(ctx, image, k, ptrs, ms, ns, st, _mode(mode), C.byref(p), out),
           "zts_search_batch_pruned")
    return [r.as_dict() for r in out]


class DeviceBatch:
    """Argument arrays of zts_search_batch_pruned_device for a fixed list of device templates (built once, so
    a loop that searches the same templates repeatedly marshals nothing per call)."""

    def __init__(self, tensors):
        self.tensors = list(tensors)
        k = len(self.tensors)
        self.count = k
        self.ptrs = (C.c_void_p * k)(*[t.data_ptr() for t in self.tensors])
        self.ms = (C.c_int32 * k)(*[t.shape[0] for t in self.tensors])
        self.ns = (C.c_int32 * k)(*[t.shape[1] for t in self.tensors])
        self.st = (C.c_int64 * k)(*[t.stride(0) for t in self.tensors])
        self.out = (Result * k)()


def zts_search_batch_pruned_device(ctx, image: int, batch: DeviceBatch, mode, params: Params | None = None,
                                   stream=None):
    """zts_search_batch_pruned on device templates (read in place after the caller's stream); fills and
    returns batch.out (a ctypes array of Result)."""
    p = params if params is not None else zts_params_default()
    s = stream if stream is not None else _current_stream(batch.tensors[0].device.index)
    _check(lib().zts_search_batch_pruned_device(ctx, image, batch.count, batch.ptrs, batch.ms, batch.ns, batch.st,
                                                _mode(mode), C.byref(p), s, batch.out),
           "zts_search_batch_pruned_device")
    return batch.out


def _tpl_arrays(tpls):
    tpls = [_u8(t) for t in tpls]
    k = len(tpls)
    ptrs = (C.c_void_p * k)(*[t.ctypes.data for t in tpls])
    ms = (C.c_int32 * k)(*[t.shape[0] for t in tpls])
    ns = (C.c_int32 * k)(*[t.shape[1] for t in tpls])
    st = (C.c_int64 * k)(*[t.strides[0] for t in tpls])
    return tpls, ptrs, ms, ns, st


def zts_submit(ctx, image: int, tpl, mode, params: Params | None = None) -> int:
    """Queues one search; returns its ticket (the template is copied before returning)."""
    tpl = _u8(tpl)
    p = params if params is not None else zts_params_default()
    t = C.c_uint64()
    _check(lib().zts_submit(ctx, image, tpl.ctypes.data, tpl.shape[0], tpl.shape[1], tpl.strides[0], _mode(mode),
                            C.byref(p), C.byref(t)), "zts_submit")
    return t.value


def zts_submit_batch(ctx, image: int, tpls, mode, params: Params | None = None) -> list:
    tpls, ptrs, ms, ns, st = _tpl_arrays(tpls)
    p = params if params is not None else zts_params_default()
    t = C.c_uint64()
    _check(lib().zts_submit_batch(ctx, image, len(tpls), ptrs, ms, ns, st, _mode(mode), C.byref(p), C.byref(t)),
           "zts_submit_batch")
    return list(range(t.value, t.value + len(tpls)))


def zts_poll(ctx, ticket: int):
    """None while the request runs; then (status, result dict)."""
    r = Result()
    rc = lib().zts_poll(ctx, ticket, C.byref(r))
    if rc == -6:
        return None
    if rc == -1:
        raise ZtsError(rc, "zts_poll")
    return rc, r.as_dict()


def zts_wait(ctx, ticket: int, timeout_ns: int = -1):
    """(status, result dict) once the request has ended; raises ZtsError(-8) on time-out."""
    r = Result()
    rc = lib().zts_wait(ctx, ticket, timeout_ns, C.byref(r))
    if rc in (-1, -8):
        raise ZtsError(rc, "zts_wait")
    return rc, r.as_dict()


def zts_cancel(ctx, ticket: int) -> None:
    _check(lib().zts_cancel(ctx, ticket), "zts_cancel")


def zts_pending(ctx):
    q, r = C.c_int32(), C.c_int32()
    _check(lib().zts_pending(ctx, C.byref(q), C.byref(r)), "zts_pending")
    return q.value, r.value


def zts_debug_full_map(ctx, image: int, image_shape, tpl):
    tpl = _u8(tpl)
    Ly, Lx = image_shape[0] - tpl.shape[0] + 1, image_shape[1] - tpl.shape[1] + 1
    if Ly < 1 or Lx < 1:
        raise ZtsError(-2, "zts_debug_full_map")
    num = np.zeros((Ly, Lx), np.int64)
    dr = np.zeros((Ly, Lx), np.int64)
    rho = np.zeros((Ly, Lx), np.float32)
    _check(lib().zts_debug_full_map(ctx, image, tpl.ctypes.data, tpl.shape[0], tpl.shape[1], tpl.strides[0],
                                    num.ctypes.data, dr.ctypes.data, rho.ctypes.data), "zts_debug_full_map")
    return num, dr, rho


def zts_debug_autocorr(ctx, image: int, image_shape, m: int, n: int, h: int, w: int):
    Ly, Lx = image_shape[0] - m + 1, image_shape[1] - n + 1
    if Ly < 1 or Lx < 1:
        raise ZtsError(-2, "zts_debug_autocorr")
    arrs = [np.zeros(Ly * Lx, np.int64) for _ in range(3)]
    _check(lib().zts_debug_autocorr(ctx, image, m, n, h, w, *(a.ctypes.data for a in arrs)), "zts_debug_autocorr")
    return tuple(arrs)


def zts_debug_blur(ctx, img, taps) -> np.ndarray:
    img = np.ascontiguousarray(_u8(img))
    taps = np.ascontiguousarray(taps, np.int32)
    d = (len(taps) - 1) // 2
    out = np.zeros_like(img)
    _check(lib().zts_debug_blur(ctx, img.ctypes.data, img.shape[0], img.shape[1], taps.ctypes.data, d,
                                out.ctypes.data), "zts_debug_blur")
    return out


class Searcher:
    """Convenience owner of one context: load images, search templates."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_inflight: int = 0, max_queued: int = 0,
                 tune_cache: str | None = None):
        self.ctx = zts_create(device, hbm_budget_bytes, max_inflight, max_queued, tune_cache)
        self.shapes = {}

    def close(self):
        if self.ctx:
            zts_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, img) -> int:
        img = _u8(img)
        i = zts_image_load(self.ctx, img)
        self.shapes[i] = img.shape
        return i

    def load_device(self, tensor) -> int:
        i = zts_image_load_device(self.ctx, tensor)
        self.shapes[i] = tuple(tensor.shape)
        return i

    def unload(self, image):
        zts_image_unload(self.ctx, image)
        self.shapes.pop(image, None)

    def prepare(self, image, m, n, mode, **params):
        zts_prepare(self.ctx, image, m, n, mode, zts_params_default(**params))
        if _mode(mode) not in (ZTS_FULL, ZTS_FULL_MFMA):
            return zts_prep_query(self.ctx, image, m, n, mode)
        return None

    def search(self, image, tpl, mode="egs", decision=False, **params):
        p = zts_params_default(**params)
        if decision:
            return zts_search_decision(self.ctx, image, self.shapes[image], tpl, mode, p)
        return zts_search(self.ctx, image, tpl, mode, p)

    def search_batch(self, image, tpls):
        return zts_search_batch(self.ctx, image, tpls)

    def search_batch_pruned(self, image, tpls, mode="opta", **params):
        return zts_search_batch_pruned(self.ctx, image, tpls, mode, zts_params_default(**params))

    def tune_batch(self, image, sizes):
        return zts_tune_batch(self.ctx, image, sizes)

    def submit(self, image, tpl, mode="full_mfma", **params):
        return zts_submit(self.ctx, image, tpl, mode, zts_params_default(**params))

    def submit_batch(self, image, tpls, mode="full_mfma", **params):
        return zts_submit_batch(self.ctx, image, tpls, mode, zts_params_default(**params))

    def poll(self, ticket):
        return zts_poll(self.ctx, ticket)

    def wait(self, ticket, timeout_ns=-1):
        return zts_wait(self.ctx, ticket, timeout_ns)

    def cancel(self, ticket):
        zts_cancel(self.ctx, ticket)

    def pending(self):
        return zts_pending(self.ctx)

    def prep_image(self, image, m, n, mode="opta"):
        return zts_prep_image(self.ctx, image, m, n, self.shapes[image], mode)
