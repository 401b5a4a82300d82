"""Python view of the CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain, single-threaded C implementation of qdot written from
the paper (arXiv 2105.00115), plus an exact FP64 dot product.  Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It never imports the device library and the
device library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

KMIN, KMAX = -2148, 2047
W = KMAX - KMIN + 1
DOUBLE, SINGLE, HALF, PERF = 0, 1, 2, 3
F_UNATTAINABLE, F_THM_ALL_DOUBLE, F_ALL_PERF, F_OVERFLOW = 1, 2, 4, 8
F_GUARANTEED, F_RESELECTED = 16, 32
OK, E_INVAL, E_NONFINITE, E_BREAKDOWN, E_MAXIT = 0, 1, 2, 5, 6


class OrcResult(C.Structure):
    _fields_ = [
        ("value", C.c_double),
        ("count", C.c_int64 * 4),
        ("n_zero", C.c_int64),
        ("e_min", C.c_int32),
        ("e_max", C.c_int32),
        ("n_bins", C.c_int32),
        ("t", C.c_int32),
        ("part", C.c_double * 3),
        ("bound_rel", C.c_double),
        ("bound_abs", C.c_double),
        ("bound_rig", C.c_double),
        ("flags", C.c_int32),
        ("status", C.c_int32),
        ("lower", C.c_double),
        ("e_ref", C.c_int32),
        ("passes", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {
            "value": self.value,
            "count": list(self.count),
            "n_zero": self.n_zero,
            "e_min": self.e_min,
            "e_max": self.e_max,
            "n_bins": self.n_bins,
            "t": self.t,
            "part": list(self.part),
            "bound_rel": self.bound_rel,
            "bound_abs": self.bound_abs,
            "bound_rig": self.bound_rig,
            "flags": self.flags,
            "status": self.status,
            "lower": self.lower,
            "e_ref": self.e_ref,
            "passes": self.passes,
        }


_lib = None

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)
_fp = C.POINTER(C.c_float)
_fp = C.POINTER(C.c_float)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    L = C.CDLL(_build.LIB)
    L.orc_qdot.argtypes = [_dp, _dp, C.c_int64, C.c_double, _i32p,
                           C.POINTER(OrcResult), _u8p, _i32p, _i64p]
    L.orc_qdot.restype = C.c_int
    L.orc_qdot_f32.argtypes = [_fp, _fp, C.c_int64, C.c_double, _i32p,
                               C.POINTER(OrcResult), _u8p, _i32p, _i64p]
    L.orc_qdot_f32.restype = C.c_int
    for f in ("orc_dot_exact", "orc_abs_dot", "orc_dot_dot2"):
        getattr(L, f).argtypes = [_dp, _dp, C.c_int64]
        getattr(L, f).restype = C.c_double
    L.orc_sum_exact.argtypes = [_dp, C.c_int64]
    L.orc_sum_exact.restype = C.c_double
    L.orc_split.argtypes = [C.c_double, _i32p, _dp]
    L.orc_split.restype = None
    L.orc_key.argtypes = [C.c_double, C.c_double, C.c_int32]
    L.orc_key.restype = C.c_int32
    L.orc_r16.argtypes = [C.c_double]
    L.orc_r16.restype = C.c_double
    L.orc_t.argtypes = [C.c_int64, C.c_double]
    L.orc_t.restype = C.c_int32
    L.orc_ceil_log2.argtypes = [C.c_int64]
    L.orc_ceil_log2.restype = C.c_int32
    L.orc_precision.argtypes = [C.c_int32, C.c_int32]
    L.orc_precision.restype = C.c_int32
    L.orc_tree64.argtypes = [_fp]
    L.orc_tree64.restype = C.c_float
    L.orc_spmv.argtypes = [C.c_int64, _i32p, _i32p, _dp, _dp, _dp]
    L.orc_spmv.restype = None
    L.orc_cg.argtypes = [C.c_int64, _i32p, _i32p, _dp, _dp, _dp, C.c_double,
                         C.c_double, C.c_int32, C.c_int32, _i32p, _i32p, _dp,
                         _dp, C.POINTER(OrcResult)]
    L.orc_cg.restype = C.c_int
    L.orc_power.argtypes = [C.c_int64, _i32p, _i32p, _dp, _dp, C.c_int32,
                            C.c_double, C.c_int32, _i32p, _dp, _dp, C.POINTER(OrcResult)]
    L.orc_power.restype = C.c_int
    _lib = L
    return L


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _opts(opt):
    if opt is None:
        return None, None
    o = np.zeros(7, dtype=np.int32)
    v = np.asarray(opt, dtype=np.int32).ravel()
    # {key, score, boundary, accum[, guard[, bin_mode, bin_param]]}
    assert v.shape[0] in (4, 5, 7)
    o[:v.shape[0]] = v
    return o, o.ctypes.data_as(_i32p)


def _qdot(fn, dtype, ptype, x, y, tol, opt, want_classes, want_keys, want_hist):
    x = np.ascontiguousarray(x, dtype=dtype)
    y = np.ascontiguousarray(y, dtype=dtype)
    assert x.shape == y.shape
    n = x.shape[0]
    o, op = _opts(opt)
    r = OrcResult()
    cls = np.zeros(n, dtype=np.uint8) if want_classes else None
    keys = np.zeros(n, dtype=np.int32) if want_keys else None
    hist = np.zeros(W, dtype=np.int64) if want_hist else None
    fn(x.ctypes.data_as(ptype), y.ctypes.data_as(ptype), n, float(tol), op, C.byref(r),
       cls.ctypes.data_as(_u8p) if cls is not None else None,
       keys.ctypes.data_as(_i32p) if keys is not None else None,
       hist.ctypes.data_as(_i64p) if hist is not None else None)
    d = r.as_dict()
    if cls is not None:
        d["classes"] = cls
    if keys is not None:
        d["keys"] = keys
    if hist is not None:
        d["hist"] = hist
    return d


def qdot(x, y, tol, opt=None, want_classes=False, want_keys=False,
         want_hist=False) -> dict:
    """Oracle qdot.  Returns the result dict, plus 'classes' (uint8[n]),
    'keys' (int32[n], zero products = INT32_MIN) and 'hist' (int64[W],
    index k - KMIN) when asked."""
    return _qdot(lib().orc_qdot, np.float64, _dp, x, y, tol, opt, want_classes, want_keys,
                 want_hist)


def qdot_f32(x, y, tol, opt=None, want_classes=False, want_keys=False,
             want_hist=False) -> dict:
    """Oracle qdot of single-precision inputs (mu = m_single): as qdot, with
    no double class."""
    return _qdot(lib().orc_qdot_f32, np.float32, _fp, x, y, tol, opt, want_classes, want_keys,
                 want_hist)


def dot_exact(x, y) -> float:
    x, xp = _f64(x)
    y, yp = _f64(y)
    return lib().orc_dot_exact(xp, yp, x.shape[0])


def dot_dot2(x, y) -> float:
    """Ogita-Rump-Oishi Dot2 compensated dot (published algorithm)."""
    x, xp = _f64(x)
    y, yp = _f64(y)
    return lib().orc_dot_dot2(xp, yp, len(x))


def bound_thm34(r: dict, exact: float):
    """A-posteriori form of the bound (Thm 3.4): with E = flexp(exact dot),
    sum_k M_k 2^(k - E + 1) eps(class_k) = bound_rel * 2^(e_max - E); the
    theorem needs e_max <= E (returned as hyp)."""
    import math
    if exact == 0.0 or r["n_bins"] == 0:
        return {"hyp": False, "bound_thm3_rel": math.inf}
    E = math.frexp(abs(exact))[1] - 1
    return {"hyp": r["e_max"] <= E, "bound_thm3_rel": math.ldexp(r["bound_rel"], r["e_max"] - E)}


def abs_dot(x, y) -> float:
    x, xp = _f64(x)
    y, yp = _f64(y)
    return lib().orc_abs_dot(xp, yp, x.shape[0])


def sum_exact(v) -> float:
    v, vp = _f64(v)
    return lib().orc_sum_exact(vp, v.shape[0])


def split(v: float):
    E = C.c_int32()
    m = C.c_double()
    lib().orc_split(float(v), C.byref(E), C.byref(m))
    return E.value, m.value


def key(x: float, y: float, key_mode: int = 0) -> int:
    return lib().orc_key(float(x), float(y), int(key_mode))


def r16(m: float) -> float:
    return lib().orc_r16(float(m))


def t_of(n_bins: int, eps: float) -> int:
    return lib().orc_t(int(n_bins), float(eps))


def ceil_log2(m: int) -> int:
    return lib().orc_ceil_log2(int(m))


def precision(sigma: int, nonstrict: int = 0) -> int:
    return lib().orc_precision(int(sigma), int(nonstrict))


def tree64(leaves) -> float:
    a = np.ascontiguousarray(leaves, dtype=np.float32)
    assert a.shape == (64,)
    return lib().orc_tree64(a.ctypes.data_as(_fp))


def _csr(rowptr, col, val):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float64)
    return rp, cl, vl


def spmv(rowptr, col, val, x):
    rp, cl, vl = _csr(rowptr, col, val)
    x, xp = _f64(x)
    out = np.empty(rp.shape[0] - 1, dtype=np.float64)
    lib().orc_spmv(out.shape[0], rp.ctypes.data_as(_i32p),
                   cl.ctypes.data_as(_i32p), vl.ctypes.data_as(_dp), xp,
                   out.ctypes.data_as(_dp))
    return out


def cg(rowptr, col, val, b, rtol, qtol, maxit, use_qdot, opt=None, x0=None,
       want_trace=False) -> dict:
    rp, cl, vl = _csr(rowptr, col, val)
    n = rp.shape[0] - 1
    b, bp = _f64(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    o, op = _opts(opt)
    it = C.c_int32()
    est = C.c_double()
    tru = C.c_double()
    trace = (OrcResult * (2 * maxit + 1))() if want_trace else None
    st = lib().orc_cg(n, rp.ctypes.data_as(_i32p), cl.ctypes.data_as(_i32p),
                      vl.ctypes.data_as(_dp), bp, x.ctypes.data_as(_dp),
                      float(rtol), float(qtol), int(maxit), int(use_qdot), op,
                      C.byref(it), C.byref(est), C.byref(tru), trace)
    d = {"status": st, "iters": it.value, "relres_est": est.value,
         "relres_true": tru.value, "x": x}
    if want_trace:
        ncalls = 1 + 2 * it.value
        d["trace"] = [trace[i].as_dict() for i in range(min(ncalls, len(trace)))]
    return d


def power(rowptr, col, val, x0, iters, qtol, use_qdot, opt=None,
          want_results=False) -> dict:
    """Oracle power method.  'trace' holds every lambda; with want_results,
    'results' holds the two inner-product results of every iteration
    (lambda's first), as many as were computed."""
    rp, cl, vl = _csr(rowptr, col, val)
    n = rp.shape[0] - 1
    x = np.array(x0, dtype=np.float64)
    o, op = _opts(opt)
    lam = C.c_double()
    tr = np.zeros(max(iters, 1), dtype=np.float64)
    res = (OrcResult * max(2 * iters, 1))() if want_results else None
    st = lib().orc_power(n, rp.ctypes.data_as(_i32p), cl.ctypes.data_as(_i32p),
                         vl.ctypes.data_as(_dp), x.ctypes.data_as(_dp),
                         int(iters), float(qtol), int(use_qdot), op,
                         C.byref(lam), tr.ctypes.data_as(_dp), res)
    d = {"status": st, "lambda": lam.value, "trace": tr[:iters], "x": x}
    if want_results:
        d["results"] = [res[i].as_dict() for i in range(2 * iters)]
    return d
