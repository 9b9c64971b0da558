"""ctypes binding of ``libkrr.so`` (the C ABI declared in ``include/krr.h``).

Argument marshalling only: every computation runs in the HIP library.  PyTorch
supplies device memory and the stream.  The library is loaded lazily; if it is
missing the first call raises ``RuntimeError`` (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkrr.so")

KRR_FP64, KRR_FP32, KRR_BF16 = 0, 1, 2
PREC = {"fp64": KRR_FP64, "fp32": KRR_FP32, "bf16": KRR_BF16}
KRR_OK, KRR_NOT_CONVERGED, KRR_BREAKDOWN = 0, 1, 2
KRR_EINVAL, KRR_ENONFINITE, KRR_EWORKSPACE, KRR_EHIP, KRR_EUNSUPPORTED = -1, -2, -3, -4, -5
KRR_INNER_CG, KRR_INNER_NONE = 0, 1
KRR_GS_MGS, KRR_GS_CGS2 = 0, 1
KRR_KERNEL_GAUSS, KRR_KERNEL_MATERN32 = 0, 1
KERNEL = {"gauss": KRR_KERNEL_GAUSS, "matern32": KRR_KERNEL_MATERN32}
KRR_MODE_FGMRES, KRR_MODE_CG64, KRR_MODE_GMRES, KRR_MODE_FCG = 0, 1, 2, 3
(KRR_WS_KMVP, KRR_WS_KMVP_MULTI, KRR_WS_KMVP_GRAD, KRR_WS_CG_INNER, KRR_WS_FGMRES, KRR_WS_SOLVE,
 KRR_WS_KMVP_CROSS, KRR_WS_PREDICT) = range(8)
KRR_MAX_DIM = 64

EXPORTED = ("krr_default_opts", "krr_status_string", "krr_workspace_size", "kmvp_gauss", "kmvp_matern",
            "kmvp_gauss_multi", "kmvp_gauss_cross", "kmvp_grad", "cg_inner_solve", "fgmres_solve",
            "krr_solve", "krr_predict", "krr_profile_begin", "krr_profile_end", "krr_probe_workspace_size",
            "krr_probe_issue_rates", "krr_lanczos_extremes", "kmvp_gauss_noalloc", "krr_noalloc_scratch_bytes")


class Points(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("x", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("restart_m", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("tol", ctypes.c_double),
                ("inner", ctypes.c_int32), ("inner_prec", ctypes.c_int32), ("delta", ctypes.c_double),
                ("inner_maxit", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("gs", ctypes.c_int32),
                ("cg_check", ctypes.c_int32), ("kernel", ctypes.c_int32)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("pairs", ctypes.c_double),
                ("pairs_skipped", ctypes.c_double)]


class ProfileStats(ctypes.Structure):
    _fields_ = [("prec", ProfileEntry * 3), ("dropped", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("mvp64", ctypes.c_int64), ("mvp32", ctypes.c_int64), ("mvp16", ctypes.c_int64),
                ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("lambda_min_est", ctypes.c_double),
                ("lambda_max_est", ctypes.c_double), ("t_prep_ms", ctypes.c_double),
                ("t_inner_ms", ctypes.c_double), ("t_outer_ms", ctypes.c_double),
                ("t_ortho_ms", ctypes.c_double), ("batch_steps", ctypes.c_int32),
                ("batch_tiles", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_P = ctypes.POINTER

_lib = None
_lock = threading.Lock()


def load(path: str | None = None):
    """Load libkrr.so and declare every exported signature."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
        lib = ctypes.CDLL(p)
        lib.krr_default_opts.argtypes = [_P(Opts)]
        lib.krr_default_opts.restype = None
        lib.krr_status_string.argtypes = [ctypes.c_int]
        lib.krr_status_string.restype = ctypes.c_char_p
        lib.krr_workspace_size.argtypes = [_i32, _P(Points), _i32, _i32, _P(Opts)]
        lib.krr_workspace_size.restype = _sz
        lib.kmvp_gauss.argtypes = [_P(Points), _dbl, _dbl, _i32, _vp, _vp, _vp, _sz, _vp]
        lib.kmvp_matern.argtypes = [_P(Points), _dbl, _dbl, _i32, _vp, _vp, _vp, _sz, _vp]
        lib.kmvp_gauss_multi.argtypes = [_P(Points), _dbl, _dbl, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _sz, _vp]
        lib.kmvp_gauss_cross.argtypes = [_P(Points), _P(Points), _dbl, _i32, _vp, _vp, _vp, _sz, _vp]
        lib.kmvp_grad.argtypes = [_P(Points), _dbl, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        lib.cg_inner_solve.argtypes = [_P(Points), _dbl, _dbl, _i32, _vp, _vp, _i32, _dbl, _P(Info), _vp, _sz, _vp]
        lib.fgmres_solve.argtypes = [_P(Points), _dbl, _dbl, _vp, _vp, _P(Opts), _P(Info), _vp, _sz, _vp]
        lib.krr_solve.argtypes = [_P(Points), _i32, _P(_dbl), _P(_dbl), _i32, _P(_vp), _P(_i64), _P(_vp), _i32,
                                  _P(Opts), _P(Info), _vp, _sz, _vp]
        lib.krr_predict.argtypes = [_P(Points), _P(Points), _dbl, _dbl, _vp, _vp, _vp, _P(Opts), _P(Info), _vp, _sz,
                                    _vp]
        lib.krr_predict.restype = ctypes.c_int
        lib.krr_profile_begin.argtypes = [_i32]
        lib.krr_profile_begin.restype = ctypes.c_int
        lib.krr_profile_end.argtypes = [_P(ProfileStats)]
        lib.krr_probe_workspace_size.restype = _sz
        lib.krr_probe_workspace_size.argtypes = []
        lib.krr_probe_issue_rates.restype = ctypes.c_int
        lib.krr_probe_issue_rates.argtypes = [_P(_dbl), _vp, _sz, _vp]
        lib.krr_lanczos_extremes.restype = ctypes.c_int
        lib.krr_lanczos_extremes.argtypes = [_P(_dbl), _P(_dbl), _i32, _P(_dbl), _P(_dbl)]
        lib.krr_profile_end.restype = ctypes.c_int
        lib.kmvp_gauss_noalloc.argtypes = [_P(Points), _dbl, _dbl, _i32, _vp, _vp, _vp]
        lib.krr_noalloc_scratch_bytes.argtypes = []
        lib.krr_noalloc_scratch_bytes.restype = _sz
        for name in ("kmvp_gauss", "kmvp_matern", "kmvp_gauss_multi", "kmvp_gauss_cross", "kmvp_grad", "cg_inner_solve",
                     "fgmres_solve", "krr_solve", "kmvp_gauss_noalloc"):
            getattr(lib, name).restype = ctypes.c_int
        if path is None:
            _lib = lib
        return lib


def status_string(code: int) -> str:
    return load().krr_status_string(int(code)).decode()


def default_opts() -> Opts:
    o = Opts()
    load().krr_default_opts(ctypes.byref(o))
    return o


def workspace_size(which: int, shapes, nrhs: int = 1, opts: Opts | None = None) -> int:
    """Workspace bytes for call `which` over point-set shapes [(n, d), ...]."""
    arr = (Points * len(shapes))(*[Points(int(n), int(d), None) for n, d in shapes])
    return int(load().krr_workspace_size(which, arr, len(shapes), int(nrhs),
                                         ctypes.byref(opts) if opts is not None else None))


class KrrError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code


def check(code: int, where: str, ok_positive: bool = True) -> int:
    if code < 0 or (code > 0 and not ok_positive):
        raise KrrError(code, where)
    return code


class profile:
    """Context manager timing every kernel-product launch (HIP events) made inside it."""

    def __init__(self, max_launches: int = 65536):
        self.max_launches = max_launches
        self.stats = None

    def __enter__(self):
        check(load().krr_profile_begin(self.max_launches), "krr_profile_begin")
        return self

    def __exit__(self, *exc):
        st = ProfileStats()
        check(load().krr_profile_end(ctypes.byref(st)), "krr_profile_end")
        names = ("fp64", "fp32", "bf16")
        self.stats = {names[k]: dict(launches=st.prec[k].launches, total_ms=st.prec[k].total_ms,
                                     pairs=st.prec[k].pairs, pairs_skipped=st.prec[k].pairs_skipped)
                      for k in range(3)}
        self.stats["dropped"] = st.dropped
        return False
