"""Python face of the CPU oracle (ctypes over ``zncc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg; never by the product library.  The
C source is compiled with gcc (``-ffp-contract=off``) into
``oracle/liboracle.so``; :func:`build` does that and the loader calls it when
the shared object is missing or older than the source.

All arrays are numpy; images and templates are uint8, 2-D, any row stride.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "zncc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class Result(C.Structure):
    _fields_ = [
        ("y", C.c_int32), ("x", C.c_int32), ("rho", C.c_double),
        ("num", C.c_int64), ("den_t", C.c_int64), ("den_r", C.c_int64),
        ("n_locations", C.c_int64), ("n_centres", C.c_int64), ("n_eliminated", C.c_int64),
        ("n_survivors", C.c_int64), ("n_computed", C.c_int64),
        ("group_h", C.c_int32), ("group_w", C.c_int32),
        ("best0", C.c_double), ("best0_y", C.c_int32), ("best0_x", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EgsStep(C.Structure):
    _fields_ = [("h", C.c_int32), ("w", C.c_int32), ("cc", C.c_int64), ("cr", C.c_int64),
                ("ct", C.c_int64), ("accepted", C.c_int32)]


class OptaParams(C.Structure):
    _fields_ = [("rho_th", C.c_double), ("rho_max", C.c_double), ("xi", C.c_double),
                ("h0", C.c_int32), ("w0", C.c_int32), ("dh", C.c_int32), ("dw", C.c_int32),
                ("hmax", C.c_int32), ("blur_kind", C.c_int32), ("sigma_step", C.c_double),
                ("sigma_max", C.c_double), ("max_iters", C.c_int32), ("nthreads", C.c_int32),
                ("paper", C.c_int32), ("estimate", C.c_int32), ("rho_tc", C.c_double), ("shape", C.c_int32),
                ("accept_xi", C.c_double)]


class OptaStep(C.Structure):
    _fields_ = [("k", C.c_int32), ("d", C.c_int32), ("passes", C.c_int32), ("h", C.c_int32),
                ("w", C.c_int32), ("accepted", C.c_int32), ("sigma", C.c_double),
                ("reverted", C.c_int64), ("cost", C.c_int64)]


ERRORS = {-1: "argument", -2: "size", -3: "degenerate template", -11: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc; returns the path of the shared object."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-pthread", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.orc_rho.restype = C.c_double
        L.orc_rho.argtypes = [C.c_int64] * 3
        L.orc_sin.restype = C.c_double
        L.orc_sin.argtypes = [C.c_int64] * 3
        L.orc_rho_twopass.restype = C.c_double
        L.orc_rho_twopass.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int, C.c_int]
        L.orc_transitive_bounds.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double),
                                            C.POINTER(C.c_double)]
        L.orc_transitive_gap.restype = C.c_double
        L.orc_transitive_gap.argtypes = [C.c_double, C.c_double]
        L.orc_lambda.restype = C.c_double
        L.orc_lambda.argtypes = [C.c_double, C.c_double]
        L.orc_ub_general.restype = C.c_int
        L.orc_ub_general.argtypes = [C.c_double] * 6 + [C.POINTER(C.c_double)]
        L.orc_location_stats.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int,
                                         _i64p, _i64p, _i64p]
        L.orc_location_stats_rs.argtypes = L.orc_location_stats.argtypes
        L.orc_full_search.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int, C.c_int,
                                      C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(Result)]
        L.orc_centre_of.restype = C.c_int64
        L.orc_centre_of.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64]
        L.orc_group_count.restype = C.c_int64
        L.orc_group_count.argtypes = [C.c_int] * 4
        L.orc_autocorr_direct.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                          C.c_int, _i64p, _i64p, _i64p]
        L.orc_autocorr_lsa.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.c_int, _i64p, _i64p, _i64p]
        L.orc_te_search.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int, C.c_int,
                                    C.c_int64, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _i64p, _i64p,
                                    _i64p,
                                    C.c_int, C.c_void_p, C.POINTER(Result)]
        L.orc_blurcorr.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int,
                                   _i64p, _i64p, _i64p]
        L.orc_gauss_taps.argtypes = [C.c_double, C.c_void_p, C.c_int, C.POINTER(C.c_int)]
        L.orc_blur.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int, C.c_void_p,
                               C.c_int64]
        L.orc_revert.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int,
                                 C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int64)]
        L.orc_egs.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                              C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(EgsStep), C.c_int,
                              C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int64)]
        L.orc_opta.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int,
                               C.POINTER(OptaParams), C.c_void_p, C.POINTER(OptaStep), C.c_int,
                               C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int64), C.POINTER(C.c_int)]
        L.orc_opta_search.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int,
                                      C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _i64p,
                                      _i64p,
                                      _i64p, _i64p, _i64p, _i64p, C.c_int, C.c_void_p, C.POINTER(Result)]
        L.orc_window_search.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_int, C.c_int,
                                        C.c_int64, C.c_int, C.c_int, C.c_int, C.POINTER(Result)]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def _u8(a):
    a = np.asarray(a)
    if a.dtype != np.uint8 or a.ndim != 2:
        raise TypeError("expected a 2-D uint8 array")
    if a.strides[1] != 1:
        a = np.ascontiguousarray(a)
    return a


def default_threads() -> int:
    return max(1, min(64, os.cpu_count() or 1))


# ---- scalars -------------------------------------------------------------

def rho(num, da, db) -> float:
    return lib().orc_rho(int(num), int(da), int(db))


def sin(num, da, db) -> float:
    return lib().orc_sin(int(num), int(da), int(db))


def rho_twopass(a, b) -> float:
    a, b = _u8(a), _u8(b)
    assert a.shape == b.shape
    return lib().orc_rho_twopass(a.ctypes.data, a.strides[0], b.ctypes.data, b.strides[0], *a.shape)


def transitive_bounds(rtc, rco):
    lb, ub = C.c_double(), C.c_double()
    lib().orc_transitive_bounds(rtc, rco, C.byref(lb), C.byref(ub))
    return lb.value, ub.value


def transitive_gap(rtc, rco) -> float:
    return lib().orc_transitive_gap(rtc, rco)


def lambda_(rho_th, rho_max) -> float:
    return lib().orc_lambda(rho_th, rho_max)


def ub_general(ra, sa, rb, sb, rc, sc):
    """(bounded, ub) of the angle-triangle bound; bounded False means no bound below 1."""
    ub = C.c_double(0.0)
    ok = lib().orc_ub_general(ra, sa, rb, sb, rc, sc, C.byref(ub))
    return bool(ok), ub.value


# ---- statistics ------------------------------------------------------------

def location_stats(img, m, n, running_sums=False):
    img = _u8(img)
    p, q = img.shape
    L = (p - m + 1) * (q - n + 1)
    S, S2, D = (np.zeros(L, np.int64) for _ in range(3))
    f = lib().orc_location_stats_rs if running_sums else lib().orc_location_stats
    _check(f(img.ctypes.data, p, q, img.strides[0], m, n, S, S2, D))
    shape = (p - m + 1, q - n + 1)
    return S.reshape(shape), S2.reshape(shape), D.reshape(shape)


def full_search(img, tpl, nthreads=None, maps=False):
    img, tpl = _u8(img), _u8(tpl)
    p, q = img.shape
    m, n = tpl.shape
    if m > p or n > q:
        raise OracleError(-2)
    L = (p - m + 1) * (q - n + 1)
    res = Result()
    arrs = [np.zeros(L, np.int64), np.zeros(L, np.int64), np.zeros(L, np.int64), np.zeros(L, np.float64)] \
        if maps else [None] * 4
    ptrs = [a.ctypes.data if a is not None else None for a in arrs]
    _check(lib().orc_full_search(img.ctypes.data, p, q, img.strides[0], tpl.ctypes.data, m, n, tpl.strides[0],
                                 nthreads or default_threads(), *ptrs, C.byref(res)))
    out = res.as_dict()
    if maps:
        shape = (p - m + 1, q - n + 1)
        out["xs_map"], out["num_map"], out["dr_map"], out["rho_map"] = (a.reshape(shape) for a in arrs)
    return out


def centre_of(Ly, Lx, h, w, l) -> int:
    return lib().orc_centre_of(Ly, Lx, h, w, l)


def group_count(Ly, Lx, h, w) -> int:
    return lib().orc_group_count(Ly, Lx, h, w)


def autocorr(img, m, n, h, w, method="lsa", nthreads=None):
    """(num, dc, do) flat int64 arrays over the location grid."""
    img = _u8(img)
    p, q = img.shape
    L = (p - m + 1) * (q - n + 1)
    num, dc, do = (np.zeros(L, np.int64) for _ in range(3))
    if method == "direct":
        _check(lib().orc_autocorr_direct(img.ctypes.data, p, q, img.strides[0], m, n, h, w, num, dc, do))
    else:
        _check(lib().orc_autocorr_lsa(img.ctypes.data, p, q, img.strides[0], m, n, h, w,
                                      nthreads or default_threads(), num, dc, do))
    return num, dc, do


def te_search(img, tpl, h, w, delta=1e-9, ac=None, decision=False, nthreads=None, radius=0, floor=-2.0):
    img, tpl = _u8(img), _u8(tpl)
    p, q = img.shape
    m, n = tpl.shape
    if ac is None:
        ac = autocorr(img, m, n, h, w, nthreads=nthreads)
    L = (p - m + 1) * (q - n + 1)
    dec = np.zeros(L, np.int8) if decision else None
    res = Result()
    _check(lib().orc_te_search(img.ctypes.data, p, q, img.strides[0], tpl.ctypes.data, m, n, tpl.strides[0],
                               h, w, delta, float(floor), radius, ac[0], ac[1], ac[2], nthreads or default_threads(),
                               dec.ctypes.data if dec is not None else None, C.byref(res)))
    out = res.as_dict()
    if decision:
        out["decision"] = dec.reshape(p - m + 1, q - n + 1)
    return out


def blurcorr(I, J, m, n):
    I, J = _u8(I), _u8(J)
    if I.strides[0] != J.strides[0]:
        I, J = np.ascontiguousarray(I), np.ascontiguousarray(J)
    p, q = I.shape
    L = (p - m + 1) * (q - n + 1)
    num, dj, di = (np.zeros(L, np.int64) for _ in range(3))
    _check(lib().orc_blurcorr(I.ctypes.data, J.ctypes.data, p, q, I.strides[0], m, n, num, dj, di))
    return num, dj, di


def gauss_taps(sigma):
    taps = np.zeros(129, np.int32)
    d = C.c_int()
    _check(lib().orc_gauss_taps(float(sigma), taps.ctypes.data, 129, C.byref(d)))
    return taps[:2 * d.value + 1].copy(), d.value


PAPER_W = np.array([1, 4, 10, 4, 1], np.int32)


def blur(img, taps):
    img = _u8(img)
    taps = np.ascontiguousarray(taps, np.int32)
    d = (len(taps) - 1) // 2
    p, q = img.shape
    out = np.zeros((p, q), np.uint8)
    _check(lib().orc_blur(img.ctypes.data, p, q, img.strides[0], taps.ctypes.data, d, out.ctypes.data, q))
    return out


def revert(I, J, m, n, lam):
    """Returns (J_after, passes, reverted_pixels); J itself is not modified."""
    I = np.ascontiguousarray(_u8(I))
    J2 = np.ascontiguousarray(_u8(J)).copy()
    p, q = I.shape
    passes, rev = C.c_int(), C.c_int64()
    _check(lib().orc_revert(I.ctypes.data, J2.ctypes.data, p, q, q, m, n, lam, C.byref(passes), C.byref(rev)))
    return J2, passes.value, rev.value


def egs(img, m, n, h0=3, w0=3, dh=2, dw=2, hmax=33, rho_th=0.8, xi=0.005, c=None, estimate=0, rho_tc=0.0, shape=0,
        nthreads=None):
    """Alg. 2.  estimate 0: Prop. 3.2 / Eq. 15; 1: Prop. 3.1 (Eq. 7, both roots) at an assumed rho_tc.
    shape 0: square steps as printed; 1: the cheapest of (h+dh, w), (h, w+dw), (h+dh, w+dw) each step.
    c: blur correlation (num, dj, di) of the searched image against the original (the exact OptA count)."""
    img = _u8(img)
    p, q = img.shape
    trace = (EgsStep * 64)()
    nt, he, we, cost = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
    cp = [a.ctypes.data for a in c] if c is not None else [None, None, None]
    _check(lib().orc_egs(img.ctypes.data, p, q, img.strides[0], m, n, h0, w0, dh, dw, hmax, rho_th, xi, *cp,
                         estimate, float(rho_tc), shape, nthreads or default_threads(), trace, 64, C.byref(nt),
                         C.byref(he), C.byref(we), C.byref(cost)))
    tr = [dict(h=s.h, w=s.w, cc=s.cc, cr=s.cr, ct=s.ct, accepted=bool(s.accepted)) for s in trace[:nt.value]]
    return {"h": he.value, "w": we.value, "cost": cost.value, "trace": tr}


def opta_params(rho_th=0.8, rho_max=0.95, xi=0.005, h0=3, w0=3, dh=2, dw=2, hmax=33, blur_kind=1,
                sigma_step=0.5, sigma_max=3.0, max_iters=6, nthreads=None, paper=False, estimate=0, rho_tc=0.0,
                shape=0, accept_xi=0.005):
    return OptaParams(rho_th, rho_max, xi, h0, w0, dh, dw, hmax, blur_kind, sigma_step, sigma_max, max_iters,
                      nthreads or default_threads(), int(bool(paper)), estimate, float(rho_tc), shape,
                      float(accept_xi))


def opta(I, m, n, **kw):
    """Alg. 3.  paper=False: the exact search's conditioning (EGS counts add each location's angle to its
    original block); paper=True: Alg. 3 as printed (EGS on each blurred image alone, Prop. 3.2)."""
    I = _u8(I)
    p, q = I.shape
    pr = opta_params(**kw)
    out = np.zeros((p, q), np.uint8)
    trace = (OptaStep * 64)()
    nt, he, we, rad = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    cost = C.c_int64()
    _check(lib().orc_opta(I.ctypes.data, p, q, I.strides[0], m, n, C.byref(pr), out.ctypes.data, trace, 64,
                          C.byref(nt), C.byref(he), C.byref(we), C.byref(cost), C.byref(rad)))
    tr = [dict(k=s.k, d=s.d, sigma=s.sigma, passes=s.passes, reverted=s.reverted, h=s.h, w=s.w, cost=s.cost,
               accepted=bool(s.accepted)) for s in trace[:nt.value]]
    return {"image": out, "h": he.value, "w": we.value, "cost": cost.value, "radius": rad.value, "trace": tr}


def opta_search(I, J, tpl, h, w, radius, delta=1e-9, decision=False, nthreads=None, floor=-2.0):
    I, J, tpl = (np.ascontiguousarray(_u8(a)) for a in (I, J, tpl))
    p, q = I.shape
    m, n = tpl.shape
    b = autocorr(J, m, n, h, w, nthreads=nthreads)
    c = blurcorr(I, J, m, n)
    L = (p - m + 1) * (q - n + 1)
    dec = np.zeros(L, np.int8) if decision else None
    res = Result()
    _check(lib().orc_opta_search(I.ctypes.data, J.ctypes.data, p, q, q, tpl.ctypes.data, m, n, n, h, w, radius,
                                 delta, float(floor), b[0], b[1], b[2], c[0], c[1], c[2], nthreads or default_threads(),
                                 dec.ctypes.data if dec is not None else None, C.byref(res)))
    out = res.as_dict()
    if decision:
        out["decision"] = dec.reshape(p - m + 1, q - n + 1)
    return out


def window_search(img, tpl, cy, cx, radius):
    """Section IV-C's localisation stage: the best of the locations within Chebyshev distance `radius` of
    (cy, cx), matched by the plain definition (C1)."""
    img, tpl = _u8(img), _u8(tpl)
    p, q = img.shape
    m, n = tpl.shape
    res = Result()
    _check(lib().orc_window_search(img.ctypes.data, p, q, img.strides[0], tpl.ctypes.data, m, n, tpl.strides[0],
                                   int(cy), int(cx), int(radius), C.byref(res)))
    return res.as_dict()


def opta_paper_search(I, J, tpl, h, w, radius, delta=1e-9, nthreads=None, floor=-2.0):
    """The paper's own OptA search (sections IV-C, V and VI, Alg. 3): transitive elimination on the
    conditioned image J with J's auto-correlation and the two-scan threshold, which finds J's best
    location exactly, then the localisation window on I around it.  Not exact on I when blurring moved or
    suppressed the peak (section V reports offsets of up to 4 pixels).  Counts: those of the search on J;
    n_computed adds the window's matches.  blurred = J's best (y, x, rho)."""
    te = te_search(J, tpl, h, w, delta=delta, nthreads=nthreads, floor=floor)
    win = window_search(I, tpl, te["y"], te["x"], radius)
    out = dict(win)
    out.update(n_centres=te["n_centres"], n_eliminated=te["n_eliminated"], n_survivors=te["n_survivors"],
               n_computed=te["n_computed"] + win["n_computed"], n_window=win["n_computed"],
               group_h=te["group_h"], group_w=te["group_w"], best0=te["best0"], best0_y=te["best0_y"],
               best0_x=te["best0_x"], blurred=(te["y"], te["x"], te["rho"]))
    return out
