"""ctypes binding of libqtprod.so: the C-ABI of include/qtprod.h, same names.

Argument marshalling only.  Pointers are plain integers (device addresses),
streams are hipStream_t handles as integers (0 = null stream).  Loading fails
loudly if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

# QTPROD_LIB selects another build of the same library (the host-sanitized
# build of the argument-validation tests); default: the in-tree library.
LIB_PATH = os.environ.get("QTPROD_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "libqtprod.so")

QT_OK = 0
QT_ERR_INVALID_ARG = -1
QT_ERR_UNSUPPORTED = -2
QT_ERR_ALLOC = -3
QT_ERR_HIP = -4
QT_ERR_TOO_LARGE = -5

QT_FP32 = 0
QT_SPLIT_BF16 = 1
QT_SPLIT_FP16 = 2
QT_FP64 = 3

QT_MAX_P = 4096
QT_NOALLOC_SCRATCH_BYTES = 256 << 20

PRECISIONS = {"fp32": QT_FP32, "split_bf16": QT_SPLIT_BF16, "split_fp16": QT_SPLIT_FP16,
              "fp64": QT_FP64}


class qt_problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("s", ctypes.c_int), ("p", ctypes.c_int),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p)]


_I, _SZ, _P = ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p

# name -> (restype, argtypes); every symbol declared in include/qtprod.h
SIGNATURES = {
    "qt_version": (_I, []),
    "qt_status_string": (ctypes.c_char_p, [_I]),
    "qt_prepare": (_I, [_I, _P]),
    "qt_fourier_ld": (_I, [_I]),
    "qt_tube_fft": (_I, [_I, _I, _I, _P, _I, _P, _I, _I, _I, _P]),
    "qt_fourier_tprod": (_I, [_I, _I, _I, _I, _P, _I, _P, _I, _P, _I, _I, _P]),
    "qt_split_words": (_I, [_I, _I, _I, _P, _I, _P]),
    "qt_workspace_size": (_SZ, [_I, _I, _I, _I, _I]),
    "qt_tprod": (_I, [_I, _I, _I, _I, _P, _P, _P, _I, _P, _SZ, _P]),
    "qt_tprod_noalloc": (_I, [_I, _I, _I, _I, _P, _P, _P, _I, _P]),
    "qt_batched_workspace_size": (_SZ, [_I, ctypes.POINTER(qt_problem), _I]),
    "qt_tprod_batched": (_I, [_I, ctypes.POINTER(qt_problem), _I, _P, _SZ, _P]),
    "qt_batched_plan_create": (_I, [_I, ctypes.POINTER(qt_problem), _I, _P, _SZ, _P,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "qt_batched_plan_launch": (_I, [_P, _P]),
    "qt_batched_plan_destroy": (_I, [_P]),
    "qt_autotune": (_I, [_I, _P]),
    "qt_complex_workspace_size": (_SZ, [_I, _I, _I, _I, _I]),
    "qt_tprod_complex": (_I, [_I, _I, _I, _I, _P, _P, _P, _I, _P, _SZ, _P]),
    "qt_real_workspace_size": (_SZ, [_I, _I, _I, _I, _I]),
    "qt_tprod_real": (_I, [_I, _I, _I, _I, _P, _P, _P, _I, _P, _SZ, _P]),
    "qt_backward_workspace_size": (_SZ, [_I, _I, _I, _I, _I]),
    "qt_tprod_backward": (_I, [_I, _I, _I, _I, _P, _P, _P, _P, _P, _I, _P, _SZ, _P]),
    "qt_tsvd_workspace_size": (_SZ, [_I, _I, _I, _I]),
    "qt_tsvd": (_I, [_I, _I, _I, _P, _P, _P, _P, _P, _I, _P, _SZ, _P]),
    "qt_fourier_tsvd_workspace_size": (_SZ, [_I, _I, _I, _I]),
    "qt_fourier_tsvd": (_I, [_I, _I, _I, _P, _I, _P, _I, _P, _I, _P, _I, _P, _SZ, _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (built beforehand by paper_2212_14318_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2212_14318_amd.build` "
                "(there is no fallback implementation)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class QtError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {qt_status_string(status)} ({status})")


def check(status: int, where: str) -> None:
    if status != QT_OK:
        raise QtError(status, where)


# ---- same-name wrappers -----------------------------------------------------

def qt_version() -> int:
    return lib().qt_version()


def qt_status_string(status: int) -> str:
    return lib().qt_status_string(status).decode()


def qt_prepare(p: int, stream: int = 0) -> int:
    return lib().qt_prepare(p, stream)


def qt_fourier_ld(cols: int) -> int:
    return lib().qt_fourier_ld(cols)


def qt_tube_fft(rows, cols, p, X, ldx, Xh, ldh, inverse, precision, stream=0) -> int:
    return lib().qt_tube_fft(rows, cols, p, X, ldx, Xh, ldh, inverse, precision, stream)


def qt_fourier_tprod(m, n, s, p, Ah, lda, Bh, ldb, Ch, ldc, precision, stream=0) -> int:
    return lib().qt_fourier_tprod(m, n, s, p, Ah, lda, Bh, ldb, Ch, ldc, precision, stream)


def qt_complex_workspace_size(m, n, s, p, precision) -> int:
    return lib().qt_complex_workspace_size(m, n, s, p, precision)


def qt_tprod_complex(m, n, s, p, A, B, C, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_tprod_complex(m, n, s, p, A, B, C, precision, ws, ws_bytes, stream)


def qt_real_workspace_size(m, n, s, p, precision) -> int:
    return lib().qt_real_workspace_size(m, n, s, p, precision)


def qt_tprod_real(m, n, s, p, A, B, C, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_tprod_real(m, n, s, p, A, B, C, precision, ws, ws_bytes, stream)


def qt_split_words(rows, cols, p, Xh, ld, stream=0) -> int:
    return lib().qt_split_words(rows, cols, p, Xh, ld, stream)


def qt_workspace_size(m: int, n: int, s: int, p: int, precision: int) -> int:
    return lib().qt_workspace_size(m, n, s, p, precision)


def qt_tprod(m, n, s, p, A, B, C, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_tprod(m, n, s, p, A, B, C, precision, ws, ws_bytes, stream)


def qt_tprod_noalloc(m, n, s, p, A, B, C, precision, stream=0) -> int:
    return lib().qt_tprod_noalloc(m, n, s, p, A, B, C, precision, stream)


def make_problems(items):
    """items: sequence of (m, n, s, p, A_ptr, B_ptr, C_ptr) -> ctypes array."""
    arr = (qt_problem * len(items))()
    for k, (m, n, s, p, a, b, c) in enumerate(items):
        arr[k] = qt_problem(m, n, s, p, a, b, c)
    return arr


def qt_batched_workspace_size(count, probs, precision) -> int:
    return lib().qt_batched_workspace_size(count, probs, precision)


def qt_tprod_batched(count, probs, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_tprod_batched(count, probs, precision, ws, ws_bytes, stream)


def qt_batched_plan_create(count, probs, precision, ws, ws_bytes, stream=0):
    """Returns (status, plan handle as int or None)."""
    h = ctypes.c_void_p()
    st = lib().qt_batched_plan_create(count, probs, precision, ws, ws_bytes, stream, ctypes.byref(h))
    return st, h.value


def qt_batched_plan_launch(plan, stream=0) -> int:
    return lib().qt_batched_plan_launch(plan, stream)


def qt_batched_plan_destroy(plan) -> int:
    return lib().qt_batched_plan_destroy(plan)


def qt_autotune(precision, stream=0) -> int:
    return lib().qt_autotune(precision, stream)


def qt_backward_workspace_size(m, n, s, p, precision) -> int:
    return lib().qt_backward_workspace_size(m, n, s, p, precision)


def qt_tprod_backward(m, n, s, p, A, B, G, dA, dB, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_tprod_backward(m, n, s, p, A, B, G, dA, dB, precision, ws, ws_bytes, stream)


def qt_tsvd_workspace_size(m, n, p, precision) -> int:
    return lib().qt_tsvd_workspace_size(m, n, p, precision)


def qt_tsvd(m, n, p, A, U, S, V, sigma, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_tsvd(m, n, p, A, U, S, V, sigma, precision, ws, ws_bytes, stream)


def qt_fourier_tsvd_workspace_size(m, n, p, precision) -> int:
    return lib().qt_fourier_tsvd_workspace_size(m, n, p, precision)


def qt_fourier_tsvd(m, n, p, Ah, lda, Uh, ldu, Vh, ldv, sigma, precision, ws, ws_bytes, stream=0) -> int:
    return lib().qt_fourier_tsvd(m, n, p, Ah, lda, Uh, ldu, Vh, ldv, sigma, precision, ws, ws_bytes, stream)
