"""ctypes binding of libtsne_mi355x.so: the C ABI declared in include/tsne_mi355x.h.

Argument marshalling only.  Loading fails loudly when the library has not
been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsne_mi355x.so")

TSNE_OK = 0
TSNE_ERR_INVALID_ARG = 1
TSNE_ERR_UNSUPPORTED = 2
TSNE_ERR_WORKSPACE = 3
TSNE_ERR_HIP = 4
TSNE_ERR_NONFINITE = 5
TSNE_ERR_SCRATCH = 6
TSNE_ABI_VERSION = 3
TSNE_KNN_FP32 = 0
TSNE_KNN_BF16 = 1
TSNE_F32 = 0
TSNE_F64 = 1
TSNE_MAX_K = 256

_p = C.c_void_p
_i64 = C.c_int64
_i32 = C.c_int32
_f32 = C.c_float
_szp = C.POINTER(C.c_size_t)


class Schedule(C.Structure):
    """tsne_schedule (include/tsne_mi355x.h)."""

    _fields_ = [("lr", C.c_float), ("exaggeration", C.c_float), ("exaggeration_iters", C.c_int32),
                ("momentum_early", C.c_float), ("momentum_late", C.c_float), ("gain_inc", C.c_float),
                ("gain_dec", C.c_float), ("min_gain", C.c_float)]


# name -> (restype, argtypes), in header order
SIGNATURES = {
    "tsne_abi_version": (C.c_int, []),
    "tsne_status_string": (C.c_char_p, [C.c_int]),
    "tsne_last_hip_error": (C.c_int, []),
    "tsne_knn": (C.c_int, [_p, _i64, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _szp, _p]),
    "tsne_calibrate_P": (C.c_int, [_p, _i64, _i32, _f32, _f32, _i32, _p, _p, _p, _p, _p]),
    "tsne_symmetrize": (C.c_int, [_p, _p, _i64, _i32, _p, _p, _p, _p, _p, _p, _szp, _p]),
    "tsne_kl_grad": (C.c_int, [_p, _i64, _p, _p, _p, _f32, _p, _p, _p, _p, _p, _p, _szp, _p]),
    "tsne_kl_grad_noalloc": (C.c_int, [_p, _i64, _p, _p, _p, _f32, _p, _p, _p, _p, _p, _p]),
    "tsne_kl_grad_fft": (C.c_int, [_p, _i64, _p, _p, _p, _f32, _i32, _i32, _f32, _i32, _p, _p, _p, _p, _p, _szp,
                                   _p]),
    "tsne_pca": (C.c_int, [_p, _i64, _i32, _i32, _i32, _p, _p, _p, _p, _p, _p, _szp, _p]),
    "tsne_step": (C.c_int, [_p, _p, _p, _p, _i64, _f32, _f32, _f32, _f32, _f32, _p]),
    "tsne_optimize": (C.c_int, [_p, _p, _p, _i64, _p, _p, _p, _i64, _i32, _i32, C.POINTER(Schedule), _i32, _p, _p,
                                _p, _p, _szp, _p]),
    "tsne_kl_forward": (C.c_int, [_i32, _p, _i64, _p, _p, _p, _p, _p, _p, _szp, _p]),
    "tsne_kl_backward": (C.c_int, [_i32, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _szp, _p]),
    "tsne_umap_fit_ab": (C.c_int, [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "tsne_umap_weights": (C.c_int, [_p, _i64, _i32, _p, _p, _p, _p]),
    "tsne_umap_fuzzy_union": (C.c_int, [_p, _p, _i64, _i32, _p, _p, _p, _p, _p, _p, _szp, _p]),
    "tsne_umap_layout": (C.c_int, [_p, _i64, _p, _p, _p, _i64, _i32, C.c_double, C.c_double, C.c_double, _i32, _i32,
                                   _i32, _i32, C.c_uint64, _p, _szp, _p]),
    "tsne_monitor_start": (C.c_int, [C.c_double, _i32, _i32, C.c_char_p, C.c_char_p, C.POINTER(C.c_void_p)]),
    "tsne_monitor_timestamp": (C.c_int, [_p, C.c_char_p]),
    "tsne_monitor_has_gpu": (C.c_int, [_p]),
    "tsne_monitor_stop": (C.c_int, [_p]),
    "tsne_monitor_steps": (C.c_int, [_p, _p, _i64, _i32, _p, _i64, _p, _p, _p]),
}

_lib = None


class TsneError(RuntimeError):
    def __init__(self, fn: str, status: int):
        lib = load()
        msg = lib.tsne_status_string(status).decode()
        extra = f" (hipError {lib.tsne_last_hip_error()})" if status == TSNE_ERR_HIP else ""
        super().__init__(f"{fn} failed: {msg}{extra}")
        self.status = status


def load():
    """Load the HIP library (once).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -m paper_2605_13928_amd.build` (no CPU fallback exists)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        if lib.tsne_abi_version() != TSNE_ABI_VERSION:
            raise RuntimeError("libtsne_mi355x ABI version mismatch")
        _lib = lib
    return _lib


def check(fn: str, status: int):
    if status != TSNE_OK:
        raise TsneError(fn, status)
