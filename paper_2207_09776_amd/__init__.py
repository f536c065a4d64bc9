"""Python binding of libmagnus (include/magnus.h): the iterated stochastic
Magnus scheme of arXiv 2207.09776 on MI355X (gfx950).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory and the current HIP stream.  Importing works
without a GPU; calling a compute function needs the built library
(``python -m paper_2207_09776_amd.build``) and a GPU, and raises otherwise.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import sys
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmagnus.so")

MG_OK, MG_EINVAL, MG_ESHAPE, MG_EUNSUPPORTED, MG_EHIP, MG_ENOMEM = 0, -1, -2, -3, -4, -5
MG_ENONFINITE = -6
MG_FLAG_NONFINITE, MG_FLAG_NORM, MG_FLAG_ABORT, MG_FLAG_NEGATIVE = 1, 2, 4, 8
MG_FP64, MG_FP32C = 0, 1
PRECISIONS = {"fp64": MG_FP64, "fp32c": MG_FP32C}

EXPORTS = ("mg_build_operators", "mg_free_operators", "mg_iterated_integrals",
           "mg_workspace_bytes", "mg_magnus_expmv", "mg_magnus_expmv_noalloc",
           "mg_workspace_bytes_multi",
           "mg_magnus_expmv_multi", "mg_autotune_expmv", "mg_autotune_cache_save",
           "mg_autotune_cache_load", "mg_select_magnus_steps",
           "mg_select_magnus_steps_per_path", "mg_iterated_integrals_steps",
           "mg_magnus_adaptive",
           "mg_euler_increments",
           "mg_euler_workspace_bytes",
           "mg_euler_step",
           "mg_error_vs_exact", "mg_check_flags",
           "mg_last_error", "mg_timing_enable", "mg_timing_read", "mg_timing_reset", "mg_version")


class MagnusError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class mg_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nv", ctypes.c_int32), ("ax", ctypes.c_double),
                ("bx", ctypes.c_double), ("av", ctypes.c_double), ("bv", ctypes.c_double)]


class mg_coeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.POINTER(ctypes.c_double))
                for n in ("h", "fx", "fv", "gxx", "gxv", "gvv", "sig", "sx", "sv")]


class mg_job(ctypes.Structure):
    _fields_ = [("ops", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("P", ctypes.c_int64),
                ("K", ctypes.c_int32), ("u0", ctypes.c_void_p), ("u0_broadcast", ctypes.c_int32),
                ("uT", ctypes.c_void_p), ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("stats", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class mg_exact(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("sigma", ctypes.c_double), ("s0sq", ctypes.c_double),
                ("T", ctypes.c_double)]


_lib = None
# bound at import: module globals (sys included) may already be None while
# objects are collected at interpreter exit
_is_finalizing = sys.is_finalizing


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmagnus.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2207_09776_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.mg_build_operators.argtypes = [ctypes.POINTER(mg_grid), ctypes.POINTER(mg_coeffs), i32,
                                       ctypes.POINTER(vp)]
    lib.mg_free_operators.argtypes = [vp]
    lib.mg_iterated_integrals.argtypes = [vp, i64, i64, dbl, i32, i32, vp, vp, vp]
    lib.mg_workspace_bytes.argtypes = [vp, i64, i32, i32]
    lib.mg_workspace_bytes.restype = sz
    lib.mg_euler_workspace_bytes.argtypes = [vp, i64]
    lib.mg_euler_workspace_bytes.restype = sz
    lib.mg_magnus_expmv.argtypes = [vp, vp, i64, i32, vp, i32, vp, i32, dbl, vp, sz, vp, vp, vp]
    lib.mg_magnus_expmv_noalloc.argtypes = [vp, vp, i64, i32, vp, i32, vp, i32, dbl, vp, vp, vp]
    lib.mg_select_magnus_steps.argtypes = [vp, vp, vp, i64, i64, dbl, vp, i32, i32, i32, dbl, i32,
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int32), vp]
    lib.mg_select_magnus_steps_per_path.argtypes = [vp, vp, vp, i64, i64, dbl, vp, i32, i32, i32,
                                                    dbl, i32, vp, vp,
                                                    ctypes.POINTER(ctypes.c_int64), vp]
    lib.mg_iterated_integrals_steps.argtypes = [vp, i64, i64, dbl, vp, i32, i32, vp, vp, vp]
    lib.mg_magnus_adaptive.argtypes = [vp, vp, vp, i64, i64, dbl, vp, i32, vp, i32, i32, i32,
                                       dbl, i32, vp, vp, vp]
    lib.mg_autotune_expmv.argtypes = [vp, vp, i64, i32, vp, i32, vp, i32, dbl, vp, sz, i32,
                                      ctypes.c_char_p, sz, vp]
    lib.mg_autotune_cache_save.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
    lib.mg_autotune_cache_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
    lib.mg_workspace_bytes_multi.argtypes = [ctypes.POINTER(mg_job), i32]
    lib.mg_workspace_bytes_multi.restype = sz
    lib.mg_magnus_expmv_multi.argtypes = [ctypes.POINTER(mg_job), i32, vp, sz, vp]
    lib.mg_euler_step.argtypes = [vp, vp, i64, vp, i32, dbl, i32, vp, sz, vp, vp]
    lib.mg_euler_increments.argtypes = [vp, i64, i64, i32, vp, vp]
    lib.mg_error_vs_exact.argtypes = [ctypes.POINTER(mg_grid), ctypes.POINTER(mg_exact), vp, vp,
                                      vp, i64, i32, vp, vp]
    lib.mg_check_flags.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i64), vp]
    lib.mg_last_error.restype = ctypes.c_char_p
    lib.mg_version.restype = ctypes.c_char_p
    lib.mg_timing_enable.argtypes = [i32]
    lib.mg_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    for name in ("mg_build_operators", "mg_free_operators", "mg_iterated_integrals",
                 "mg_magnus_expmv", "mg_magnus_expmv_noalloc", "mg_magnus_expmv_multi",
                 "mg_euler_increments",
                 "mg_euler_step", "mg_error_vs_exact", "mg_check_flags", "mg_timing_enable",
                 "mg_timing_read", "mg_timing_reset"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(code: int):
    if code != MG_OK:
        msg = load_library().mg_last_error().decode()
        raise MagnusError(code, msg)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _stream_scoped(fn):
    """Runs a binding function with the caller's stream current (see _on)."""
    import functools
    import inspect
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = sig.bind(*args, **kwargs).arguments.get("stream")
        with _on(stream):
            return fn(*args, **kwargs)
    return wrapper


@contextlib.contextmanager
def _on(stream):
    """Allocate the call's temporaries (workspace, flags, statistics) on the
    stream the library runs on: the caching allocator then reuses them only
    after the work queued there, and their zero fill is ordered before the
    kernels that write them."""
    if stream is None:
        yield
        return
    import torch
    with torch.cuda.stream(stream):
        yield


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")


class Operators:
    """mg_build_operators handle (library-owned tables on the current device)."""

    def __init__(self, nx: int, nv: int, ax: float, bx: float, av: float, bv: float,
                 coeffs: Dict[str, Optional[np.ndarray]], order: int):
        lib = load_library()
        self.grid = mg_grid(nx, nv, ax, bx, av, bv)
        self.order = order
        keep = {}
        c = mg_coeffs()
        for name, _ in mg_coeffs._fields_:
            arr = coeffs.get(name)
            if arr is None:
                setattr(c, name, None)
                continue
            a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
            if a.size != nx * nv:
                raise ValueError(f"coefficient {name} must have nx*nv entries")
            keep[name] = a
            setattr(c, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        _check(lib.mg_build_operators(ctypes.byref(self.grid), ctypes.byref(c), order,
                                      ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        """Free the library's tables now (the handle is unusable afterwards).
        The caller makes sure no queued work still uses them."""
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().mg_free_operators(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # No HIP call while the interpreter shuts down: the HIP runtime and the
        # profiler's interception may already be gone then; the process exit
        # releases the device memory.
        if _is_finalizing is None or _is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def build_operators(nx, nv, ax, bx, av, bv, coeffs, order) -> Operators:
    return Operators(nx, nv, ax, bx, av, bv, coeffs, order)


@_stream_scoped
def iterated_integrals(dW, T: float, K: int, order: int, coef=None, pathstat=None, stream=None):
    """mg_iterated_integrals: dW [P][Nf] float64 CUDA -> (coef [P][K][6], pathstat [P][2])."""
    import torch
    _dev_f64(dW, "dW")
    P, Nf = dW.shape
    if coef is None:
        coef = torch.empty((P, K, 6), dtype=torch.float64, device=dW.device)
    if pathstat is None:
        pathstat = torch.empty((P, 2), dtype=torch.float64, device=dW.device)
    _check(load_library().mg_iterated_integrals(_ptr(dW), P, Nf, float(T), K, order, _ptr(coef),
                                                _ptr(pathstat), _stream(stream)))
    return coef, pathstat


@_stream_scoped
def iterated_integrals_steps(dW, T: float, K, Kmax: int, order: int, coef=None, pathstat=None,
                             stream=None):
    """mg_iterated_integrals_steps: K int32 device [P] (steps of each path) ->
    (coef [P][Kmax][6], rows beyond K[p] zero; pathstat [P][2])."""
    import torch
    _dev_f64(dW, "dW")
    if not (K.is_cuda and K.dtype == torch.int32 and K.is_contiguous()):
        raise TypeError("K must be a contiguous int32 device tensor")
    P, Nf = dW.shape
    if K.numel() != P:
        raise ValueError("K needs one entry per path")
    if coef is None:
        coef = torch.empty((P, Kmax, 6), dtype=torch.float64, device=dW.device)
    if pathstat is None:
        pathstat = torch.empty((P, 2), dtype=torch.float64, device=dW.device)
    _check(load_library().mg_iterated_integrals_steps(_ptr(dW), P, Nf, float(T), _ptr(K), int(Kmax),
                                                      order, _ptr(coef), _ptr(pathstat),
                                                      _stream(stream)))
    return coef, pathstat


def workspace_bytes(ops: Operators, P: int, K: int, precision: str = "fp64") -> int:
    return int(load_library().mg_workspace_bytes(ops.handle, P, K, PRECISIONS[precision]))


@_stream_scoped
def magnus_expmv(ops: Operators, coef, u0, precision: str = "fp64", tol: float = 0.0,
                 uT=None, ws=None, want_stats: bool = False, stream=None):
    """mg_magnus_expmv.  u0: [N] (shared) or [P][N].  Returns (uT, flags, stats)."""
    import torch
    _dev_f64(coef, "coef")
    _dev_f64(u0, "u0")
    P, K, six = coef.shape
    N = ops.grid.nx * ops.grid.nv
    bcast = 1 if u0.dim() == 1 else 0
    if u0.numel() != (N if bcast else P * N):
        raise ValueError("u0 has the wrong size")
    dev = coef.device
    if uT is None:
        uT = torch.empty((P, N), dtype=torch.float64, device=dev)
    need = workspace_bytes(ops, P, K, precision)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    flags = torch.zeros(P, dtype=torch.int32, device=dev)
    stats = torch.zeros((P, K, 2), dtype=torch.int32, device=dev) if want_stats else None
    _check(load_library().mg_magnus_expmv(
        ops.handle, _ptr(coef), P, K, _ptr(u0), bcast, _ptr(uT), PRECISIONS[precision],
        float(tol), _ptr(ws), ws.numel(), _ptr(stats), _ptr(flags), _stream(stream)))
    return uT, flags, stats


NOALLOC_SCRATCH_BYTES = 64 << 20     # MG_NOALLOC_SCRATCH_BYTES


@_stream_scoped
def magnus_expmv_noalloc(ops: Operators, coef, u0, uT, flags=None, stats=None,
                         precision: str = "fp64", tol: float = 0.0, stream=None):
    """mg_magnus_expmv_noalloc: mg_magnus_expmv with the library's fixed
    scratch array as workspace.  The caller passes every output (uT [P][N],
    optional flags [P] int32 and stats [P][K][2] int32); nothing is allocated."""
    _dev_f64(coef, "coef")
    _dev_f64(u0, "u0")
    _dev_f64(uT, "uT")
    P, K, six = coef.shape
    N = ops.grid.nx * ops.grid.nv
    bcast = 1 if u0.dim() == 1 else 0
    if u0.numel() != (N if bcast else P * N) or uT.numel() != P * N:
        raise ValueError("u0 or uT has the wrong size")
    _check(load_library().mg_magnus_expmv_noalloc(
        ops.handle, _ptr(coef), P, K, _ptr(u0), bcast, _ptr(uT), PRECISIONS[precision],
        float(tol), _ptr(stats), _ptr(flags), _stream(stream)))
    return uT, flags, stats


@_stream_scoped
def autotune_expmv(ops: Operators, coef, u0, precision: str = "fp64", tol: float = 0.0,
                   uT=None, ws=None, reps: int = 3, stream=None) -> str:
    """mg_autotune_expmv: times the kernel shapes for this grid on the batch and
    records the fastest in ops for `precision`; returns the library's summary."""
    import torch
    _dev_f64(coef, "coef")
    _dev_f64(u0, "u0")
    P, K, six = coef.shape
    N = ops.grid.nx * ops.grid.nv
    bcast = 1 if u0.dim() == 1 else 0
    if u0.numel() != (N if bcast else P * N):
        raise ValueError("u0 has the wrong size")
    dev = coef.device
    if uT is None:
        uT = torch.empty((P, N), dtype=torch.float64, device=dev)
    if ws is None:
        ws = torch.empty(max(workspace_bytes(ops, P, K, precision), 1), dtype=torch.uint8,
                         device=dev)
    buf = ctypes.create_string_buffer(1024)
    _check(load_library().mg_autotune_expmv(
        ops.handle, _ptr(coef), P, K, _ptr(u0), bcast, _ptr(uT), PRECISIONS[precision],
        float(tol), _ptr(ws), ws.numel(), int(reps), buf, 1024, _stream(stream)))
    return buf.value.decode()


def autotune_cache_save(path: str) -> int:
    """mg_autotune_cache_save: writes the library's autotune cache; returns
    the number of entries."""
    n = ctypes.c_int32(0)
    _check(load_library().mg_autotune_cache_save(os.fsencode(path), ctypes.byref(n)))
    return int(n.value)


def autotune_cache_load(path: str) -> int:
    """mg_autotune_cache_load: merges a saved cache into the library's;
    returns the number of entries read."""
    n = ctypes.c_int32(0)
    _check(load_library().mg_autotune_cache_load(os.fsencode(path), ctypes.byref(n)))
    return int(n.value)


@_stream_scoped
def select_magnus_steps(ops2: Operators, ops3: Operators, dW, T: float, u0, K0: int,
                        factor: int = 2, Kmax: int = 1 << 20, tol: float = 1e-3,
                        precision: str = "fp64", stream=None):
    """mg_select_magnus_steps: (K, gap, accepted) from the order-2/order-3
    distance on the sample paths dW [Ps][Nf]."""
    _dev_f64(dW, "dW")
    _dev_f64(u0, "u0")
    Ps, Nf = dW.shape
    K = ctypes.c_int32(0)
    gap = ctypes.c_double(0.0)
    acc = ctypes.c_int32(0)
    _check(load_library().mg_select_magnus_steps(
        ops2.handle, ops3.handle, _ptr(dW), Ps, Nf, float(T), _ptr(u0), int(K0), int(factor),
        int(Kmax), float(tol), PRECISIONS[precision], ctypes.byref(K), ctypes.byref(gap),
        ctypes.byref(acc), _stream(stream)))
    return int(K.value), float(gap.value), bool(acc.value)


@_stream_scoped
def select_magnus_steps_per_path(ops2: Operators, ops3: Operators, dW, T: float, u0, K0: int,
                                 factor: int = 2, Kmax: int = 1 << 20, tol: float = 1e-3,
                                 precision: str = "fp64", stream=None):
    """mg_select_magnus_steps_per_path: (K [P] int32, gap [P] float64, number
    accepted) from each path's order-2/order-3 distance, dW [P][Nf]."""
    _dev_f64(dW, "dW")
    _dev_f64(u0, "u0")
    P, Nf = dW.shape
    K = np.zeros(P, dtype=np.int32)
    gap = np.zeros(P, dtype=np.float64)
    nacc = ctypes.c_int64(0)
    _check(load_library().mg_select_magnus_steps_per_path(
        ops2.handle, ops3.handle, _ptr(dW), P, Nf, float(T), _ptr(u0), int(K0), int(factor),
        int(Kmax), float(tol), PRECISIONS[precision], K.ctypes.data, gap.ctypes.data,
        ctypes.byref(nacc), _stream(stream)))
    return K, gap, int(nacc.value)


@_stream_scoped
def magnus_adaptive(ops2: Operators, ops3: Operators, dW, T: float, u0, K0: int,
                    factor: int = 2, max_level: int = 3, tol: float = 1e-3,
                    precision: str = "fp64", uT=None, stream=None):
    """mg_magnus_adaptive: (uT [P][N], level [P][K0] int32, gap [P][K0]
    float64), every coarse step of every path refined until its orders 2 and
    3 agree within tol; dW [P][Nf], u0 [N] (shared) or [P][N]."""
    import torch
    _dev_f64(dW, "dW")
    _dev_f64(u0, "u0")
    P, Nf = dW.shape
    N = ops2.grid.nx * ops2.grid.nv
    bcast = 1 if u0.dim() == 1 else 0
    if u0.numel() != (N if bcast else P * N):
        raise ValueError("u0 has the wrong size")
    if uT is None:
        uT = torch.empty((P, N), dtype=torch.float64, device=dW.device)
    level = np.zeros((P, K0), dtype=np.int32)
    gap = np.zeros((P, K0), dtype=np.float64)
    _check(load_library().mg_magnus_adaptive(
        ops2.handle, ops3.handle, _ptr(dW), P, Nf, float(T), _ptr(u0), bcast, _ptr(uT),
        int(K0), int(factor), int(max_level), float(tol), PRECISIONS[precision],
        level.ctypes.data, gap.ctypes.data, _stream(stream)))
    return uT, level, gap


def _addr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _job_array(jobs):
    arr = (mg_job * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        arr[i] = mg_job(j["ops"].handle.value, _addr(j["coef"]), j["P"], j["K"], _addr(j["u0"]),
                        j["u0_broadcast"], _addr(j["uT"]), PRECISIONS[j.get("precision", "fp64")],
                        float(j.get("tol", 0.0)), _addr(j.get("stats")), _addr(j.get("flags")))
    return arr


@_stream_scoped
def magnus_expmv_multi(jobs, ws=None, stream=None):
    """mg_magnus_expmv_multi.  Each job is a dict with ops, coef [P][K][6], u0
    ([N] or [P][N]), and optionally precision, tol, uT, want_stats; returns a
    list of (uT, flags, stats) in job order."""
    import torch
    prepared = []
    for j in jobs:
        _dev_f64(j["coef"], "coef")
        _dev_f64(j["u0"], "u0")
        P, K, _ = j["coef"].shape
        N = j["ops"].grid.nx * j["ops"].grid.nv
        bcast = 1 if j["u0"].dim() == 1 else 0
        if j["u0"].numel() != (N if bcast else P * N):
            raise ValueError("u0 has the wrong size")
        dev = j["coef"].device
        uT = j.get("uT")
        if uT is None:
            uT = torch.empty((P, N), dtype=torch.float64, device=dev)
        flags = torch.zeros(P, dtype=torch.int32, device=dev)
        stats = torch.zeros((P, K, 2), dtype=torch.int32, device=dev) if j.get("want_stats") else None
        prepared.append({"ops": j["ops"], "coef": j["coef"], "P": P, "K": K, "u0": j["u0"],
                         "u0_broadcast": bcast, "uT": uT, "precision": j.get("precision", "fp64"),
                         "tol": j.get("tol", 0.0), "stats": stats, "flags": flags})
    arr = _job_array(prepared)
    lib = load_library()
    need = int(lib.mg_workspace_bytes_multi(arr, len(prepared)))
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8,
                         device=prepared[0]["coef"].device if prepared else "cuda")
    _check(lib.mg_magnus_expmv_multi(arr, len(prepared), _ptr(ws), ws.numel(), _stream(stream)))
    return [(j["uT"], j["flags"], j["stats"]) for j in prepared]


@_stream_scoped
def euler_increments(dW, NE: int, dWE=None, stream=None):
    """mg_euler_increments: [P][Nf] fine increments -> [P][NE] Euler increments."""
    import torch
    _dev_f64(dW, "dW")
    P, Nf = dW.shape
    if dWE is None:
        dWE = torch.empty((P, NE), dtype=torch.float64, device=dW.device)
    _check(load_library().mg_euler_increments(_ptr(dW), P, Nf, NE, _ptr(dWE), _stream(stream)))
    return dWE


def euler_workspace_bytes(ops: Operators, P: int) -> int:
    """mg_euler_workspace_bytes (raises MagnusError if no Euler kernel fits)."""
    n = int(load_library().mg_euler_workspace_bytes(ops.handle, P))
    if n == ctypes.c_size_t(-1).value:
        raise MagnusError(MG_EUNSUPPORTED, "mg_euler_workspace_bytes: no Euler kernel for this grid")
    return n


@_stream_scoped
def euler_step(ops: Operators, u, dWE, dt: float, ws=None, stream=None):
    """mg_euler_step: NE Euler-Maruyama steps in place on u [P][N]; returns flags."""
    import torch
    _dev_f64(u, "u")
    _dev_f64(dWE, "dWE")
    P, NE = dWE.shape
    flags = torch.zeros(P, dtype=torch.int32, device=u.device)
    if ws is None:
        need = euler_workspace_bytes(ops, P)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=u.device) if need else None
    _check(load_library().mg_euler_step(ops.handle, _ptr(u), P, _ptr(dWE), NE, float(dt), MG_FP64,
                                        _ptr(ws) if ws is not None else None,
                                        ws.numel() if ws is not None else 0, _ptr(flags),
                                        _stream(stream)))
    return flags


@_stream_scoped
def error_vs_exact(ops_or_grid, u, pathstat=None, a=None, sigma=None, s0sq=None, T=None,
                   uref=None, kappa: int = 0, err=None, stream=None):
    """mg_error_vs_exact: per-path relative Frobenius error on the kappa window."""
    import torch
    grid = ops_or_grid.grid if isinstance(ops_or_grid, Operators) else ops_or_grid
    _dev_f64(u, "u")
    P = u.shape[0]
    if err is None:
        err = torch.empty(P, dtype=torch.float64, device=u.device)
    ex = None
    if uref is None:
        _dev_f64(pathstat, "pathstat")
        ex = mg_exact(a, sigma, s0sq, T)
    else:
        _dev_f64(uref, "uref")
    _check(load_library().mg_error_vs_exact(
        ctypes.byref(grid), ctypes.byref(ex) if ex is not None else None, _ptr(pathstat), _ptr(u),
        _ptr(uref), P, kappa, _ptr(err), _stream(stream)))
    return err


@_stream_scoped
def check_flags(flags, stream=None):
    """mg_check_flags: waits for the stream; returns (OR of all flags, first
    flagged path or -1).  Raises MagnusError(MG_ENONFINITE) if any path is
    flagged."""
    import torch
    if not (isinstance(flags, torch.Tensor) and flags.is_cuda and flags.dtype == torch.int32
            and flags.is_contiguous()):
        raise TypeError("flags must be a contiguous int32 CUDA tensor")
    bits = ctypes.c_int32(0)
    first = ctypes.c_int64(-1)
    _check(load_library().mg_check_flags(_ptr(flags), flags.numel(), ctypes.byref(bits),
                                         ctypes.byref(first), _stream(stream)))
    return int(bits.value), int(first.value)


def timing_enable(on: bool = True):
    _check(load_library().mg_timing_enable(1 if on else 0))


def timing_reset():
    _check(load_library().mg_timing_reset())


def timing_read(kernel: str):
    """(total milliseconds, launches) of the named kernel since the last reset."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load_library().mg_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value
