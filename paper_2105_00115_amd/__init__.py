"""qdot on MI355X: Python binding of ``libqdot.so``.

The binding only marshals arguments: every step of qdot (exponent scan,
cutoff selection, quantised accumulation, FP64 combine) and of the CG and
power-method drivers runs in the library's HIP kernels.  PyTorch supplies
device memory and streams.  If the library has not been built, loading
fails loudly; there is no fallback.

Two layers:

* ``lib()`` -- the raw C ABI (names as in ``include/qdot.h``), taking
  integer device addresses.
* ``Qdot`` -- a handle wrapper taking torch tensors (float64, CUDA,
  contiguous) and the current torch stream.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqdot.so")

OK, E_INVAL, E_NONFINITE, E_DEVICE, E_NOMEM, E_BREAKDOWN, E_MAXIT = range(7)
DOUBLE, SINGLE, HALF, PERF = 0, 1, 2, 3
F_UNATTAINABLE, F_THM_ALL_DOUBLE, F_ALL_PERF, F_OVERFLOW = 1, 2, 4, 8
F_GUARANTEED, F_RESELECTED = 16, 32
KMIN, KMAX = -2148, 2047
W = KMAX - KMIN + 1


class QdotOptions(C.Structure):
    _fields_ = [("key_mode", C.c_int32), ("score_mode", C.c_int32),
                ("boundary_mode", C.c_int32), ("accum_mode", C.c_int32),
                ("guard_mode", C.c_int32), ("bin_mode", C.c_int32), ("bin_param", C.c_int32),
                ("tile_skip", C.c_int32)]


class QdotResult(C.Structure):
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
        ("flags", C.c_int32),
        ("status", C.c_int32),
        ("lower", C.c_double),
        ("e_ref", C.c_int32),
        ("passes", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {
            "value": self.value, "count": list(self.count), "n_zero": self.n_zero,
            "e_min": self.e_min, "e_max": self.e_max, "n_bins": self.n_bins,
            "t": self.t, "part": list(self.part), "bound_rel": self.bound_rel,
            "bound_abs": self.bound_abs, "flags": self.flags, "status": self.status,
            "lower": self.lower, "e_ref": self.e_ref, "passes": self.passes,
        }


class QdotCsr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class QdotCgResult(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32),
                ("relres_est", C.c_double), ("relres_true", C.c_double)]


class QdotCgSystem(C.Structure):
    _fields_ = [("A", QdotCsr), ("b", C.c_void_p), ("x", C.c_void_p), ("rtol", C.c_double),
                ("qtol", C.c_double), ("maxit", C.c_int32), ("use_qdot", C.c_int32)]


CG_RESULT_BYTES = C.sizeof(QdotCgResult)


class QdotTune(C.Structure):
    _fields_ = [("scan_blocks_per_cu", C.c_int32), ("scan_unroll", C.c_int32),
                ("acc_blocks_per_cu", C.c_int32), ("acc_unroll", C.c_int32),
                ("onepass_blocks_per_cu", C.c_int32), ("onepass_unroll", C.c_int32),
                ("acc_form", C.c_int32), ("hist_copies", C.c_int32),
                ("block_threads", C.c_int32)]


class QdotSolverTune(C.Structure):
    _fields_ = [("batch_blocks_per_cu", C.c_int32), ("batch_chunk", C.c_int32),
                ("cg_rows_per_block", C.c_int32), ("cg_gang_max", C.c_int32),
                ("spmv_blocks_per_cu", C.c_int32), ("cg_blocks_per_cu", C.c_int32),
                ("power_scan_in_spmv", C.c_int32)]


SOLVER_TUNE_FIELDS = tuple(f for f, _ in QdotSolverTune._fields_)


TUNE_BUCKETS = 4  # n < 2^16, < 2^20, < 2^24, >= 2^24


def tune_bucket(n: int) -> int:
    return 0 if n < 1 << 16 else 1 if n < 1 << 20 else 2 if n < 1 << 24 else 3


RESULT_BYTES = C.sizeof(QdotResult)

# (name, restype, argtypes) of every entry point in include/qdot.h
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_OPT = C.POINTER(QdotOptions)
_CSR = C.POINTER(QdotCsr)
SIGNATURES = [
    ("qdot_create", _i32, [C.POINTER(_vp), _i32]),
    ("qdot_destroy", _i32, [_vp]),
    ("qdot_last_error", C.c_char_p, [_vp]),
    ("qdot_device_info", _i32, [_vp, C.POINTER(_i32), C.POINTER(_i32)]),
    ("qdot_set_tune", _i32, [_vp, _i32, C.POINTER(QdotTune)]),
    ("qdot_get_tune", _i32, [_vp, _i32, C.POINTER(QdotTune)]),
    ("qdot_load_tune", _i32, [_vp, C.c_char_p]),
    ("qdot_timing_enable", _i32, [_vp, _i32]),
    ("qdot_timing_read", _i32, [_vp, C.POINTER(_d), C.POINTER(_i32)]),
    ("qdot_async", _i32, [_vp, _vp, _vp, _i64, _d, _OPT, _vp, _vp]),
    ("qdot", _i32, [_vp, _vp, _vp, _i64, _d, _OPT, _vp, C.POINTER(QdotResult)]),
    ("qdot_noalloc_async", _i32, [_vp, _vp, _i64, _d, _OPT, _vp, _vp]),
    ("qdot_simple", _i32, [_vp, _vp, _i64, _d, C.POINTER(_d), C.POINTER(_i64)]),
    ("qdot_classes_async", _i32, [_vp, _vp, _vp, _i64, _d, _OPT, _vp, _vp, _vp, _vp]),
    ("qdot_f32_async", _i32, [_vp, _vp, _vp, _i64, _d, _OPT, _vp, _vp]),
    ("qdot_f32", _i32, [_vp, _vp, _vp, _i64, _d, _OPT, _vp, C.POINTER(QdotResult)]),
    ("qdot_f32_classes_async", _i32, [_vp, _vp, _vp, _i64, _d, _OPT, _vp, _vp, _vp, _vp]),
    ("qdot_fp64_dot_async", _i32, [_vp, _vp, _vp, _i64, _vp, _vp]),
    ("qdot_batched_async", _i32, [_vp, _vp, _vp, _vp, C.POINTER(_i64), _vp, _i32, _OPT,
                                  _vp, _vp]),
    ("qdot_set_solver_tune", _i32, [_vp, C.POINTER(QdotSolverTune)]),
    ("qdot_get_solver_tune", _i32, [_vp, C.POINTER(QdotSolverTune)]),
    ("qdot_batched_plan", _i32, [_vp, C.POINTER(_i64), _i32]),
    ("qdot_batch_run_async", _i32, [_vp, _vp, _vp, _vp, C.POINTER(_i64), _vp, _i32,
                                    C.POINTER(QdotCgSystem), _i32, _OPT, _vp, _vp, _vp]),
    ("qdot_batch_plan", _i32, [_vp, C.POINTER(_i64), _i32, C.POINTER(QdotCgSystem), _i32,
                               _OPT]),
    ("qdot_cg_batched", _i32, [_vp, C.POINTER(QdotCgSystem), _i32, _OPT, _vp,
                               C.POINTER(QdotCgResult)]),
    ("qdot_spmv_async", _i32, [_vp, _CSR, _vp, _vp, _vp]),
    ("qdot_cg", _i32, [_vp, _CSR, _vp, _vp, _d, _d, _i32, _i32, _OPT, _vp,
                       C.POINTER(QdotCgResult), _vp]),
    ("qdot_power", _i32, [_vp, _CSR, _vp, _i32, _d, _i32, _OPT, _vp,
                          C.POINTER(_d), _vp, _vp]),
]

_lib = None


class QdotError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        super().__init__(f"{where}: status {code} {msg}".strip())
        self.code = code


def lib():
    """The loaded C library.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"qdot HIP library not found at {LIB_PATH}; build it first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch bundles its own HIP runtime under the same soname as the system
    # one the library links to; whichever is loaded first serves the whole
    # process.  Loading torch first keeps its runtime (the one its kernels
    # and allocator are built for) and binds the library to it as well.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _opts(opt):
    if opt is None:
        return None
    if isinstance(opt, QdotOptions):
        return C.byref(opt)
    if isinstance(opt, dict):
        return C.byref(QdotOptions(**opt))
    return C.byref(QdotOptions(*[int(v) for v in opt]))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_vec(t, name, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.dim() == 1):
        raise ValueError(f"{name} must be a contiguous 1-D {dtype} CUDA tensor")


def parse_cg_results(buf) -> list:
    """qdot_cg_result records from a CUDA uint8 tensor, as dicts."""
    raw = bytes(buf.cpu().numpy().tobytes())
    out = []
    for i in range(len(raw) // CG_RESULT_BYTES):
        r = QdotCgResult.from_buffer_copy(raw, i * CG_RESULT_BYTES)
        out.append({"status": r.status, "iters": r.iters, "relres_est": r.relres_est,
                    "relres_true": r.relres_true})
    return out


def parse_results(buf) -> list:
    """Decode a uint8 tensor / bytes holding one or more qdot_result."""
    raw = bytes(buf.cpu().numpy().tobytes()) if hasattr(buf, "cpu") else bytes(buf)
    n = len(raw) // RESULT_BYTES
    return [QdotResult.from_buffer_copy(raw, i * RESULT_BYTES).as_dict() for i in range(n)]


class Csr:
    """CSR matrix on the device (int32 indices, float64 values)."""

    def __init__(self, rowptr, col, val, device="cuda"):
        import torch
        self.rowptr = torch.as_tensor(rowptr, dtype=torch.int32).to(device).contiguous()
        self.col = torch.as_tensor(col, dtype=torch.int32).to(device).contiguous()
        self.val = torch.as_tensor(val, dtype=torch.float64).to(device).contiguous()
        self.n = self.rowptr.numel() - 1
        self.c = QdotCsr(self.n, self.col.numel(), self.rowptr.data_ptr(),
                         self.col.data_ptr(), self.val.data_ptr())


def qdot_simple(x, y, tol):
    """The library's minimal entry point: (value, counts) of qdot(x, y) at
    tol with default options on its own per-device handle, synchronous."""
    _check_vec(x, "x")
    _check_vec(y, "y")
    v = C.c_double()
    counts = (C.c_int64 * 4)()
    st = lib().qdot_simple(_ptr(x), _ptr(y), x.numel(), float(tol), C.byref(v), counts)
    if st not in (OK, E_NONFINITE):
        raise QdotError(st, "qdot_simple")
    return v.value, list(counts)


def qdot_noalloc_async(x, y, tol, out, opt=None, stream=None):
    """The library's allocation-free qdot (no handle; the workspace is a
    fixed device array inside the library).  out: CUDA uint8 tensor of
    RESULT_BYTES (or an integer device address), written in stream order
    on the current device."""
    _check_vec(x, "x")
    _check_vec(y, "y")
    dst = C.c_void_p(out if isinstance(out, int) else out.data_ptr())
    st = lib().qdot_noalloc_async(_ptr(x), _ptr(y), x.numel(), float(tol), _opts(opt),
                                  _stream(stream), dst)
    if st != OK:
        raise QdotError(st, "qdot_noalloc_async")


def tuned_file(device: int = 0):
    """Autotuner output for this device model, if the tuner has been run."""
    import torch
    props = torch.cuda.get_device_properties(device)
    arch = props.gcnArchName.split(":")[0]
    return os.path.join(PKG, "tune", f"{arch}_{props.multi_processor_count}cu.txt")


class Qdot:
    """A library handle bound to one device.  Loads the autotuned launch
    shapes for the device when ``tune/<arch>_<cus>cu.txt`` exists."""

    def __init__(self, device: int = 0, load_tuned: bool = True):
        self._h = C.c_void_p()
        st = lib().qdot_create(C.byref(self._h), int(device))
        if st != OK:
            raise QdotError(st, "qdot_create")
        self.device = device
        self.tune_file = None
        if load_tuned and not os.environ.get("QDOT_TUNE_FILE"):
            path = tuned_file(device)
            if path is not None and os.path.exists(path):
                self.load_tune(path)
                self.tune_file = path

    def close(self):
        if self._h:
            lib().qdot_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st, where):
        raise QdotError(st, where, lib().qdot_last_error(self._h).decode())

    # ---- configuration ----------------------------------------------------
    def device_info(self):
        d, c = C.c_int32(), C.c_int32()
        lib().qdot_device_info(self._h, C.byref(d), C.byref(c))
        return d.value, c.value

    def set_tune(self, bucket: int, scan_bpc: int, scan_unroll: int, acc_bpc: int,
                 acc_unroll: int, onepass_bpc: int = 4, onepass_unroll: int = 1,
                 acc_form: int = 0, hist_copies: int = 8, block_threads: int = 256):
        """bucket -1 sets all size buckets."""
        cfg = QdotTune(scan_bpc, scan_unroll, acc_bpc, acc_unroll, onepass_bpc, onepass_unroll,
                       acc_form, hist_copies, block_threads)
        st = lib().qdot_set_tune(self._h, int(bucket), C.byref(cfg))
        if st != OK:
            self._raise(st, "qdot_set_tune")

    def reset_tune(self):
        lib().qdot_set_tune(self._h, -1, None)

    def get_tune(self, bucket: int):
        t = QdotTune()
        st = lib().qdot_get_tune(self._h, int(bucket), C.byref(t))
        if st != OK:
            raise QdotError(st, "qdot_get_tune")
        return (t.scan_blocks_per_cu, t.scan_unroll, t.acc_blocks_per_cu, t.acc_unroll,
                t.onepass_blocks_per_cu, t.onepass_unroll, t.acc_form, t.hist_copies,
                t.block_threads)

    def set_solver_tune(self, **fields):
        """Launch shapes of the solvers and the batched launch (fields of
        QdotSolverTune); fields not given keep their values, no argument
        at all restores the defaults."""
        if not fields:
            st = lib().qdot_set_solver_tune(self._h, None)
        else:
            bad = set(fields) - set(SOLVER_TUNE_FIELDS)
            if bad:
                raise ValueError(f"unknown solver tune fields {sorted(bad)}")
            cur = dict(zip(SOLVER_TUNE_FIELDS, self.get_solver_tune()))
            cur.update({k: int(v) for k, v in fields.items()})
            cfg = QdotSolverTune(*[cur[f] for f in SOLVER_TUNE_FIELDS])
            st = lib().qdot_set_solver_tune(self._h, C.byref(cfg))
        if st != OK:
            self._raise(st, "qdot_set_solver_tune")

    def get_solver_tune(self):
        t = QdotSolverTune()
        st = lib().qdot_get_solver_tune(self._h, C.byref(t))
        if st != OK:
            raise QdotError(st, "qdot_get_solver_tune")
        return tuple(getattr(t, f) for f in SOLVER_TUNE_FIELDS)

    def load_tune(self, path: str):
        st = lib().qdot_load_tune(self._h, os.fsencode(path))
        if st != OK:
            self._raise(st, "qdot_load_tune")

    def timing_enable(self, on: bool = True):
        lib().qdot_timing_enable(self._h, 1 if on else 0)

    def timing_read(self) -> dict:
        ms = (C.c_double * 5)()
        calls = (C.c_int32 * 2)()
        st = lib().qdot_timing_read(self._h, ms, calls)
        if st != OK:
            self._raise(st, "qdot_timing_read")
        return {"scan_ms": ms[0], "cut_ms": ms[1], "acc_ms": ms[2], "fin_ms": ms[3],
                "dot64_ms": ms[4], "qdot_calls": calls[0], "dot64_calls": calls[1]}

    # ---- qdot --------------------------------------------------------------
    def qdot(self, x, y, tol, opt=None, stream=None) -> dict:
        _check_vec(x, "x")
        _check_vec(y, "y")
        r = QdotResult()
        st = lib().qdot(self._h, _ptr(x), _ptr(y), x.numel(), float(tol), _opts(opt),
                        _stream(stream), C.byref(r))
        if st not in (OK, E_NONFINITE):
            self._raise(st, "qdot")
        return r.as_dict()

    def qdot_async(self, x, y, tol, out, opt=None, stream=None):
        """out: CUDA uint8 tensor of RESULT_BYTES (or a slice address int)."""
        _check_vec(x, "x")
        _check_vec(y, "y")
        dst = C.c_void_p(out if isinstance(out, int) else out.data_ptr())
        st = lib().qdot_async(self._h, _ptr(x), _ptr(y), x.numel(), float(tol), _opts(opt),
                              _stream(stream), dst)
        if st != OK:
            self._raise(st, "qdot_async")

    def qdot_classes(self, x, y, tol, opt=None, stream=None):
        """(classes uint8[n], histogram int64[W], result dict), synchronised."""
        import torch
        _check_vec(x, "x")
        _check_vec(y, "y")
        n = x.numel()
        cls = torch.empty(max(n, 1), dtype=torch.uint8, device=x.device)
        hist = torch.empty(W, dtype=torch.int64, device=x.device)
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=x.device)
        st = lib().qdot_classes_async(self._h, _ptr(x), _ptr(y), n, float(tol), _opts(opt),
                                      _stream(stream), _ptr(cls), _ptr(hist), _ptr(out))
        if st != OK:
            self._raise(st, "qdot_classes_async")
        torch.cuda.current_stream().synchronize()
        return cls[:n], hist, parse_results(out)[0]

    # ---- single-precision inputs (mu = m_single) ----------------------------
    def qdot_f32(self, x, y, tol, opt=None, stream=None) -> dict:
        import torch
        _check_vec(x, "x", torch.float32)
        _check_vec(y, "y", torch.float32)
        r = QdotResult()
        st = lib().qdot_f32(self._h, _ptr(x), _ptr(y), x.numel(), float(tol), _opts(opt),
                            _stream(stream), C.byref(r))
        if st not in (OK, E_NONFINITE):
            self._raise(st, "qdot_f32")
        return r.as_dict()

    def qdot_f32_async(self, x, y, tol, out, opt=None, stream=None):
        import torch
        _check_vec(x, "x", torch.float32)
        _check_vec(y, "y", torch.float32)
        dst = C.c_void_p(out if isinstance(out, int) else out.data_ptr())
        st = lib().qdot_f32_async(self._h, _ptr(x), _ptr(y), x.numel(), float(tol),
                                  _opts(opt), _stream(stream), dst)
        if st != OK:
            self._raise(st, "qdot_f32_async")

    def qdot_f32_classes(self, x, y, tol, opt=None, stream=None):
        """(classes uint8[n], histogram int64[W], result dict), synchronised."""
        import torch
        _check_vec(x, "x", torch.float32)
        _check_vec(y, "y", torch.float32)
        n = x.numel()
        cls = torch.empty(max(n, 1), dtype=torch.uint8, device=x.device)
        hist = torch.empty(W, dtype=torch.int64, device=x.device)
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=x.device)
        st = lib().qdot_f32_classes_async(self._h, _ptr(x), _ptr(y), n, float(tol),
                                          _opts(opt), _stream(stream), _ptr(cls), _ptr(hist),
                                          _ptr(out))
        if st != OK:
            self._raise(st, "qdot_f32_classes_async")
        torch.cuda.current_stream().synchronize()
        return cls[:n], hist, parse_results(out)[0]

    def fp64_dot_async(self, x, y, out, stream=None):
        _check_vec(x, "x")
        _check_vec(y, "y")
        st = lib().qdot_fp64_dot_async(self._h, _ptr(x), _ptr(y), x.numel(),
                                       _stream(stream), _ptr(out))
        if st != OK:
            self._raise(st, "qdot_fp64_dot_async")

    def fp64_dot(self, x, y) -> float:
        import torch
        out = torch.empty(1, dtype=torch.float64, device=x.device)
        self.fp64_dot_async(x, y, out)
        return float(out.item())

    # ---- batched ------------------------------------------------------------
    @staticmethod
    def _host_offsets(host_offsets):
        import numpy as np
        ho = np.ascontiguousarray(host_offsets, dtype=np.int64)
        return ho, ho.ctypes.data_as(C.POINTER(C.c_int64))

    def batched_plan(self, host_offsets):
        ho, hp = self._host_offsets(host_offsets)
        st = lib().qdot_batched_plan(self._h, hp, ho.shape[0] - 1)
        if st != OK:
            self._raise(st, "qdot_batched_plan")

    def batched_async(self, x_cat, y_cat, offsets, host_offsets, tols, out, opt=None,
                      stream=None):
        """offsets (int64, B+1) and tols (float64, B) are device tensors,
        host_offsets the same offsets on the host; out is a CUDA uint8
        tensor of B * RESULT_BYTES."""
        import torch
        _check_vec(x_cat, "x_cat")
        _check_vec(y_cat, "y_cat")
        if not (offsets.is_cuda and offsets.dtype == torch.int64 and tols.is_cuda
                and tols.dtype == torch.float64):
            raise ValueError("offsets must be CUDA int64 and tols CUDA float64")
        ho, hp = self._host_offsets(host_offsets)
        B = ho.shape[0] - 1
        st = lib().qdot_batched_async(self._h, _ptr(x_cat), _ptr(y_cat), _ptr(offsets), hp,
                                      _ptr(tols), B, _opts(opt), _stream(stream), _ptr(out))
        if st != OK:
            self._raise(st, "qdot_batched_async")

    def batched(self, x_cat, y_cat, host_offsets, tols, opt=None) -> list:
        """Synchronous convenience wrapper: host offsets / tolerances."""
        import numpy as np
        import torch
        ho = np.ascontiguousarray(host_offsets, dtype=np.int64)
        dev = x_cat.device
        off_d = torch.from_numpy(ho).to(dev)
        tol_d = torch.as_tensor(np.asarray(tols, dtype=np.float64)).to(dev)
        out = torch.zeros(max(1, ho.shape[0] - 1) * RESULT_BYTES, dtype=torch.uint8, device=dev)
        self.batched_async(x_cat, y_cat, off_d, ho, tol_d, out, opt)
        torch.cuda.current_stream().synchronize()
        return parse_results(out)[: ho.shape[0] - 1]

    # ---- batched launch of qdot instances and CG systems ---------------------
    @staticmethod
    def cg_systems(systems):
        """systems: sequence of (Csr, b, x, rtol, qtol, maxit, use_qdot) with
        device tensors b, x; returns the ctypes array (keep it alive)."""
        arr = (QdotCgSystem * max(1, len(systems)))()
        for i, (A, bv, xv, rtol, qtol, maxit, use) in enumerate(systems):
            _check_vec(bv, "b")
            _check_vec(xv, "x")
            arr[i] = QdotCgSystem(A.c, bv.data_ptr(), xv.data_ptr(), float(rtol), float(qtol),
                                  int(maxit), int(use))
        return arr

    def batch_plan(self, host_offsets, systems, opt=None):
        ho, hp = self._host_offsets(host_offsets if host_offsets is not None else [0])
        arr = self.cg_systems(systems)
        st = lib().qdot_batch_plan(self._h, hp, ho.shape[0] - 1, arr, len(systems), _opts(opt))
        if st != OK:
            self._raise(st, "qdot_batch_plan")

    def batch_run_async(self, x_cat, y_cat, offsets, host_offsets, tols, out, systems,
                        cg_out, opt=None, stream=None):
        """qdot instances as batched_async (host_offsets None for none) plus
        CG systems (see cg_systems); cg_out: CUDA uint8 tensor of
        len(systems) * CG_RESULT_BYTES."""
        ho, hp = self._host_offsets(host_offsets if host_offsets is not None else [0])
        B = ho.shape[0] - 1
        arr = self.cg_systems(systems)
        st = lib().qdot_batch_run_async(
            self._h, _ptr(x_cat) if B else None, _ptr(y_cat) if B else None,
            _ptr(offsets) if B else None, hp, _ptr(tols) if B else None, B, arr, len(systems),
            _opts(opt), _stream(stream), _ptr(out) if B else None,
            _ptr(cg_out) if systems else None)
        if st != OK:
            self._raise(st, "qdot_batch_run_async")

    def cg_batched(self, systems, opt=None, stream=None) -> list:
        """Solves every system in one launch; returns one result dict each."""
        arr = self.cg_systems(systems)
        res = (QdotCgResult * max(1, len(systems)))()
        st = lib().qdot_cg_batched(self._h, arr, len(systems), _opts(opt), _stream(stream), res)
        if st != OK:
            self._raise(st, "qdot_cg_batched")
        return [{"status": r.status, "iters": r.iters, "relres_est": r.relres_est,
                 "relres_true": r.relres_true} for r in res[: len(systems)]]

    # ---- applications ------------------------------------------------------
    def spmv(self, A: Csr, x, y, stream=None):
        st = lib().qdot_spmv_async(self._h, C.byref(A.c), _ptr(x), _ptr(y), _stream(stream))
        if st != OK:
            self._raise(st, "qdot_spmv_async")

    def cg(self, A: Csr, b, x, rtol, qtol, maxit, use_qdot, opt=None, trace=False,
           stream=None) -> dict:
        import torch
        _check_vec(b, "b")
        _check_vec(x, "x")
        tr = (torch.zeros((2 * maxit + 1) * RESULT_BYTES, dtype=torch.uint8, device=b.device)
              if trace else None)
        r = QdotCgResult()
        st = lib().qdot_cg(self._h, C.byref(A.c), _ptr(b), _ptr(x), float(rtol), float(qtol),
                           int(maxit), int(use_qdot), _opts(opt), _stream(stream), C.byref(r),
                           _ptr(tr))
        if st not in (OK, E_BREAKDOWN, E_MAXIT):
            self._raise(st, "qdot_cg")
        d = {"status": r.status, "iters": r.iters, "relres_est": r.relres_est,
             "relres_true": r.relres_true}
        if trace:
            d["trace"] = parse_results(tr[: (1 + 2 * r.iters) * RESULT_BYTES])
        return d

    def power(self, A: Csr, x, iters, qtol, use_qdot, opt=None, trace=True,
              results=False, stream=None) -> dict:
        """trace: return every lambda; results: also every qdot result
        (d["results"][2k] is lambda's, [2k + 1] c's, of iteration k)."""
        import torch
        _check_vec(x, "x")
        tr = torch.zeros(max(iters, 1), dtype=torch.float64, device=x.device) if trace else None
        rs = (torch.zeros(max(2 * iters, 1) * RESULT_BYTES, dtype=torch.uint8, device=x.device)
              if results else None)
        lam = C.c_double()
        st = lib().qdot_power(self._h, C.byref(A.c), _ptr(x), int(iters), float(qtol),
                              int(use_qdot), _opts(opt), _stream(stream), C.byref(lam),
                              _ptr(tr), _ptr(rs))
        if st not in (OK, E_BREAKDOWN):
            self._raise(st, "qdot_power")
        d = {"status": st, "lambda": lam.value}
        if trace:
            d["trace"] = tr[:iters].cpu().numpy()
        if results:
            d["results"] = parse_results(rs[: 2 * iters * RESULT_BYTES])
        return d
