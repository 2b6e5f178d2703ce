"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes its workspace as documented and rejects invalid
arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_2212_14318_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtprod.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = header_functions()
    for n in ["qt_tprod", "qt_tprod_batched", "qt_tprod_backward", "qt_workspace_size",
              "qt_status_string", "qt_tube_fft"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = nat.lib()
    for name in header_functions():
        assert hasattr(lib, name), f"{name} declared in qtprod.h but not exported"
        assert name in nat.SIGNATURES, f"{name} has no Python binding"


def test_status_strings():
    for st in (nat.QT_OK, nat.QT_ERR_INVALID_ARG, nat.QT_ERR_UNSUPPORTED, nat.QT_ERR_ALLOC,
               nat.QT_ERR_HIP, nat.QT_ERR_TOO_LARGE):
        s = nat.qt_status_string(st)
        assert s.startswith("QT_")
    assert "unknown" in nat.qt_status_string(12345)
    assert nat.qt_version() >= 100


def _fourier_bytes(rows, cols, p, esize):
    ld = (cols + 3) // 4 * 4
    b = 4 * p * rows * ld * esize
    return (b + 255) // 256 * 256


@pytest.mark.parametrize("m,n,s,p", [(1, 1, 1, 1), (8, 8, 8, 8), (256, 256, 256, 64), (17, 5, 33, 7)])
def test_workspace_size_formula(m, n, s, p):
    for prec, es in ((nat.QT_FP32, 4), (nat.QT_SPLIT_BF16, 4), (nat.QT_FP64, 8)):
        want = _fourier_bytes(m, n, p, es) + _fourier_bytes(n, s, p, es) + _fourier_bytes(m, s, p, es)
        assert nat.qt_workspace_size(m, n, s, p, prec) == want


def test_workspace_size_invalid_is_zero():
    assert nat.qt_workspace_size(0, 4, 4, 4, nat.QT_FP32) == 0
    assert nat.qt_workspace_size(4, 4, 4, -1, nat.QT_FP32) == 0
    assert nat.qt_workspace_size(4, 4, 4, 4, 99) == 0


def test_workspace_size_monotone():
    prev = 0
    for m in (1, 7, 64, 100, 513):
        w = nat.qt_workspace_size(m, 33, 21, 12, nat.QT_FP32)
        assert w > prev
        prev = w


# Fake, never-dereferenced device addresses: every call below must be rejected
# on the host before the library touches HIP.
A_, B_, C_, W_ = 0x10000000, 0x20000000, 0x30000000, 0x40000000


@pytest.mark.parametrize("args", [
    (0, 4, 4, 4), (4, 0, 4, 4), (4, 4, 0, 4), (4, 4, 4, 0), (-3, 4, 4, 4),
])
def test_tprod_rejects_bad_sizes(args):
    m, n, s, p = args
    st = nat.qt_tprod(m, n, s, p, A_, B_, C_, nat.QT_FP32, W_, 1 << 30, None)
    assert st == nat.QT_ERR_INVALID_ARG


def test_tprod_rejects_null_misaligned_aliased_and_small_ws():
    ws = nat.qt_workspace_size(8, 8, 8, 8, nat.QT_FP32)
    ok = (8, 8, 8, 8)
    assert nat.qt_tprod(*ok, None, B_, C_, nat.QT_FP32, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_, None, C_, nat.QT_FP32, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_, B_, None, nat.QT_FP32, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_, B_, C_, nat.QT_FP32, None, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_ + 4, B_, C_, nat.QT_FP32, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_, B_, C_ + 8, nat.QT_FP32, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_, B_, C_, nat.QT_FP32, W_, ws - 1, None) == nat.QT_ERR_INVALID_ARG
    # C overlapping A, workspace overlapping B
    assert nat.qt_tprod(*ok, A_, B_, A_ + 256, nat.QT_FP32, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(*ok, A_, B_, C_, nat.QT_FP32, B_, ws, None) == nat.QT_ERR_INVALID_ARG
    # unknown precision
    assert nat.qt_tprod(*ok, A_, B_, C_, 7, W_, ws, None) == nat.QT_ERR_INVALID_ARG


def test_noalloc_rejects_bad_args_and_oversize_on_host():
    ok = (8, 8, 8, 8)
    F = nat.QT_FP32
    assert nat.qt_tprod_noalloc(0, 8, 8, 8, A_, B_, C_, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_noalloc(*ok, None, B_, C_, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_noalloc(*ok, A_ + 4, B_, C_, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_noalloc(*ok, A_, B_, A_ + 256, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_noalloc(*ok, A_, B_, C_, 7, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_noalloc(8, 8, 8, nat.QT_MAX_P + 1, A_, B_, C_, F, None) == nat.QT_ERR_UNSUPPORTED
    # 512^3, p = 32: 402 MB of workspace, beyond the fixed array
    big = (512, 512, 512, 32)
    assert nat.qt_workspace_size(*big, F) > nat.QT_NOALLOC_SCRATCH_BYTES
    assert nat.qt_tprod_noalloc(*big, A_, B_, C_, F, None) == nat.QT_ERR_TOO_LARGE


def test_tube_fft_rejects_bad_args():
    F = nat.QT_FP32
    assert nat.qt_tube_fft(0, 4, 4, A_, 4, B_, 4, 0, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tube_fft(4, 4, 4, A_, 4, A_ + 16, 4, 0, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tube_fft(4, 4, 4, A_, 4, B_, 4, 2, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tube_fft(4, 4, 4, A_, 3, B_, 4, 0, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tube_fft(4, 4, 4, A_, 4, B_, 3, 0, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tube_fft(4, 4, 4, A_, 4, B_, 4, 0, 9, None) == nat.QT_ERR_INVALID_ARG


def test_fourier_tprod_rejects_bad_args():
    F = nat.QT_FP32
    ok = (8, 8, 8, 8)
    assert nat.qt_fourier_tprod(*ok, A_, 6, B_, 8, C_, 8, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_fourier_tprod(*ok, A_, 8, B_, 8, C_, 7, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_fourier_tprod(*ok, A_, 10, B_, 8, C_, 8, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_fourier_tprod(*ok, A_, 8, B_, 8, A_, 8, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_fourier_tprod(0, 8, 8, 8, A_, 8, B_, 8, C_, 8, F, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_fourier_ld(5) == 8 and nat.qt_fourier_ld(8) == 8 and nat.qt_fourier_ld(0) == 0


@pytest.mark.parametrize("m,n,s,p", [(1, 1, 1, 1), (17, 5, 33, 7), (256, 256, 256, 64)])
def test_complex_workspace_formula(m, n, s, p):
    half = lambda r, c: (2 * p * r * ((c + 3) // 4 * 4) * 4 + 255) // 256 * 256
    want = half(m, n) + half(n, s) + half(m, s)
    for prec in (nat.QT_FP32, nat.QT_SPLIT_BF16):
        assert nat.qt_complex_workspace_size(m, n, s, p, prec) == want
    assert nat.qt_complex_workspace_size(m, n, s, p, nat.QT_FP64) == 0


@pytest.mark.parametrize("m,n,s,p", [(1, 1, 1, 1), (17, 5, 33, 7), (256, 256, 256, 64), (9, 9, 9, 97)])
def test_real_workspace_formula(m, n, s, p):
    h = p // 2 + 1
    part = lambda r, c: (2 * h * r * ((c + 3) // 4 * 4) * 4 + 255) // 256 * 256
    want = part(m, n) + part(n, s) + part(m, s)
    for prec in (nat.QT_FP32, nat.QT_SPLIT_BF16):
        assert nat.qt_real_workspace_size(m, n, s, p, prec) == want
    # split fp16 adds the per-frequency scales and max-abs partials
    nb = lambda r, c: min(64, (r * c + 255) // 256)
    extra = (4 * h * (2 + nb(m, n) + nb(n, s)) + 255) // 256 * 256
    assert nat.qt_real_workspace_size(m, n, s, p, nat.QT_SPLIT_FP16) == want + extra
    assert nat.qt_real_workspace_size(m, n, s, p, nat.QT_FP64) == 0


def test_real_rejects_bad_args():
    a, b, c = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
    w = ctypes.c_void_p(4 << 20)          # never dereferenced: rejected before any launch
    ws_n = nat.qt_real_workspace_size(4, 4, 4, 4, nat.QT_FP32)
    assert nat.qt_tprod_real(4, 0, 4, 4, a, b, c, nat.QT_FP32, w, ws_n, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_real(4, 4, 4, 4, a, None, c, nat.QT_FP32, w, ws_n, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_real(4, 4, 4, 4, a, b, c, nat.QT_FP64, w, ws_n, None) == nat.QT_ERR_UNSUPPORTED
    assert nat.qt_tprod_real(4, 4, 4, 4, a, b, c, nat.QT_FP32, w, ws_n - 1, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_real(4, 4, 4, 4, a, b, b, nat.QT_FP32, w, ws_n, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_real(4, 4, 4, 4, a, b, c, nat.QT_FP32, ctypes.c_void_p((4 << 20) + 4), ws_n,
                             None) == nat.QT_ERR_INVALID_ARG


def test_complex_rejects_bad_args():
    buf = ctypes.c_void_p(1 << 20)       # never dereferenced: rejected before any launch
    ws_n = nat.qt_complex_workspace_size(4, 4, 4, 4, nat.QT_FP32)
    assert nat.qt_tprod_complex(0, 4, 4, 4, buf, buf, buf, nat.QT_FP32, buf, ws_n, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_complex(4, 4, 4, 4, None, buf, buf, nat.QT_FP32, buf, ws_n, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_complex(4, 4, 4, 4, buf, buf, buf, nat.QT_FP64, buf, ws_n, None) == nat.QT_ERR_UNSUPPORTED
    assert nat.qt_tprod_complex(4, 4, 4, 4, buf, buf, buf, 9, buf, ws_n, None) == nat.QT_ERR_INVALID_ARG
    a, b, c = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
    w = ctypes.c_void_p(4 << 20)
    assert nat.qt_tprod_complex(4, 4, 4, 4, a, b, c, nat.QT_FP32, w, ws_n - 1, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_complex(4, 4, 4, 4, a, b, a, nat.QT_FP32, w, ws_n, None) == nat.QT_ERR_INVALID_ARG


def test_null_workspace_needs_zero_bytes():
    """ws == NULL asks the library to allocate, which requires ws_bytes == 0
    and a valid problem; both cases are rejected before any HIP call."""
    a, b, c = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
    g, da, db = ctypes.c_void_p(4 << 20), ctypes.c_void_p(5 << 20), ctypes.c_void_p(6 << 20)
    inv = nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod(4, 4, 4, 4, a, b, c, nat.QT_FP32, None, 64, None) == inv
    assert nat.qt_tprod(0, 4, 4, 4, a, b, c, nat.QT_FP32, None, 0, None) == inv
    assert nat.qt_tprod_complex(4, 4, 4, 4, a, b, c, nat.QT_FP32, None, 64, None) == inv
    assert nat.qt_tprod_real(4, 4, 0, 4, a, b, c, nat.QT_FP32, None, 0, None) == inv
    assert nat.qt_tprod_backward(4, 4, 4, 4, a, b, g, da, db, nat.QT_FP32, None, 64, None) == inv
    assert nat.qt_tprod_backward(4, 4, 4, 0, a, b, g, da, db, nat.QT_FP32, None, 0, None) == inv
    probs = (nat.qt_problem * 1)(nat.qt_problem(4, 4, 4, 4, a, b, c))
    assert nat.qt_tprod_batched(1, probs, nat.QT_FP32, None, 64, None) == inv
    bad = (nat.qt_problem * 1)(nat.qt_problem(0, 4, 4, 4, a, b, c))
    assert nat.qt_tprod_batched(1, bad, nat.QT_FP32, None, 0, None) == inv
    # an unsupported precision keeps its own status when the library would allocate
    uns = nat.QT_ERR_UNSUPPORTED
    assert nat.qt_tprod_complex(4, 4, 4, 4, a, b, c, nat.QT_FP64, None, 0, None) == uns
    assert nat.qt_tprod_real(4, 4, 4, 4, a, b, c, nat.QT_FP64, None, 0, None) == uns


def test_split_words_rejects_bad_args():
    buf = ctypes.c_void_p(4096)          # never dereferenced: rejected before any launch
    assert nat.qt_split_words(0, 4, 4, buf, 4, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_split_words(4, 4, 4, None, 4, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_split_words(4, 5, 4, buf, 5, None) == nat.QT_ERR_INVALID_ARG   # ld not a multiple of 4
    assert nat.qt_split_words(4, 8, 4, buf, 4, None) == nat.QT_ERR_INVALID_ARG   # ld < cols
    assert nat.qt_split_words(4, 4, 4, ctypes.c_void_p(4098), 4, None) == nat.QT_ERR_INVALID_ARG


def test_prepare_rejects_bad_p():
    assert nat.qt_prepare(0, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_prepare(nat.QT_MAX_P + 1, None) == nat.QT_ERR_UNSUPPORTED


def test_product_path_has_no_oracle_or_fallback():
    """The package never imports the oracle and has no CPU implementation."""
    pkg = os.path.join(ROOT, "paper_2212_14318_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "oracle" not in src.replace("no fallback", ""), f
            assert "numpy" not in src, f


def _tensor_bytes(rows, cols, p, esize):
    return (4 * p * rows * cols * esize + 255) // 256 * 256


@pytest.mark.parametrize("m,n,s,p", [(8, 8, 8, 8), (512, 64, 512, 100), (5, 3, 7, 2)])
def test_backward_workspace_formula(m, n, s, p):
    for prec, es in ((nat.QT_FP32, 4), (nat.QT_FP64, 8)):
        want = (_tensor_bytes(s, n, p, es) + _tensor_bytes(n, m, p, es) + _fourier_bytes(m, s, p, es)
                + _fourier_bytes(s, n, p, es) + _fourier_bytes(n, m, p, es)
                + _fourier_bytes(m, n, p, es) + _fourier_bytes(n, s, p, es))
        assert nat.qt_backward_workspace_size(m, n, s, p, prec) == want


def test_backward_rejects_bad_args():
    G_, dA_, dB_ = 0x50000000, 0x60000000, 0x70000000
    ws = nat.qt_backward_workspace_size(8, 8, 8, 8, nat.QT_FP32)
    ok = (8, 8, 8, 8)
    F = nat.QT_FP32
    assert nat.qt_tprod_backward(*ok, None, B_, G_, dA_, dB_, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_backward(*ok, A_, B_, None, dA_, dB_, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_backward(*ok, A_, B_, G_, dA_, dB_, F, W_, ws - 1, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_backward(*ok, A_, B_, G_, A_, dB_, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_backward(*ok, A_, B_, G_, dA_, G_ + 64, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_backward(*ok, A_, B_, G_, dA_ + 4, dB_, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_backward(0, 8, 8, 8, A_, B_, G_, dA_, dB_, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    # nothing requested: valid no-op without touching the device
    assert nat.qt_tprod_backward(*ok, A_, B_, G_, None, None, F, W_, ws, None) == nat.QT_OK


def test_batched_rejects_bad_args():
    F = nat.QT_FP32
    good = [(8, 8, 8, 8, A_, B_, C_)]
    probs = nat.make_problems(good)
    ws = nat.qt_batched_workspace_size(1, probs, F)
    assert ws > 0
    assert nat.qt_tprod_batched(0, probs, F, W_, ws, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_batched(1, probs, F, W_, ws - 1, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_tprod_batched(1, probs, F, None, ws, None) == nat.QT_ERR_INVALID_ARG
    bad = nat.make_problems([(0, 8, 8, 8, A_, B_, C_)])
    assert nat.qt_tprod_batched(1, bad, F, W_, 1 << 30, None) == nat.QT_ERR_INVALID_ARG
    alias = nat.make_problems([(8, 8, 8, 8, A_, B_, A_)])
    assert nat.qt_tprod_batched(1, alias, F, W_, 1 << 30, None) == nat.QT_ERR_INVALID_ARG
    # two problems writing overlapping outputs; an output overlapping another's input
    two = nat.make_problems([(8, 8, 8, 8, A_, B_, C_), (8, 8, 8, 8, A_, B_, C_ + 1024)])
    assert nat.qt_tprod_batched(2, two, F, W_, 1 << 30, None) == nat.QT_ERR_INVALID_ARG
    cross = nat.make_problems([(8, 8, 8, 8, A_, B_, C_), (8, 8, 8, 8, C_, B_, C_ + (1 << 20))])
    assert nat.qt_tprod_batched(2, cross, F, W_, 1 << 30, None) == nat.QT_ERR_INVALID_ARG
    # shared inputs are fine; p beyond QT_MAX_P or an unsupported precision is
    # reported as such (every p up to QT_MAX_P is served)
    big_p = nat.make_problems([(8, 8, 8, nat.QT_MAX_P + 1, A_, B_, C_)])
    assert nat.qt_tprod_batched(1, big_p, F, W_, 1 << 40, None) == nat.QT_ERR_UNSUPPORTED
    assert nat.qt_tprod_batched(1, probs, nat.QT_FP64, W_, 1 << 30, None) == nat.QT_ERR_UNSUPPORTED
    st, plan = nat.qt_batched_plan_create(0, probs, F, W_, ws, None)
    assert st == nat.QT_ERR_INVALID_ARG and plan is None
    assert nat.qt_batched_plan_launch(None, None) == nat.QT_ERR_INVALID_ARG
    assert nat.qt_batched_plan_destroy(None) == nat.QT_ERR_INVALID_ARG


def test_batched_workspace_size_grows():
    F = nat.QT_FP32
    one = nat.make_problems([(16, 16, 16, 8, A_, B_, C_)])
    two = nat.make_problems([(16, 16, 16, 8, A_, B_, C_), (200, 30, 70, 45, A_, B_, C_)])
    assert 0 < nat.qt_batched_workspace_size(1, one, F) < nat.qt_batched_workspace_size(2, two, F)
    assert nat.qt_batched_workspace_size(0, one, F) == 0


_FAULT_CHILD = r"""
import ctypes, sys
sys.path.insert(0, {root!r})
from paper_2212_14318_amd import _native as nat
a, b, c = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20), ctypes.c_void_p(3 << 20)
g, da, db = ctypes.c_void_p(4 << 20), ctypes.c_void_p(5 << 20), ctypes.c_void_p(6 << 20)
probs = (nat.qt_problem * 1)(nat.qt_problem(4, 4, 4, 8, a, b, c))
print(nat.qt_tprod(4, 4, 4, 8, a, b, c, nat.QT_FP32, None, 0, None),
      nat.qt_tprod_complex(4, 4, 4, 8, a, b, c, nat.QT_FP32, None, 0, None),
      nat.qt_tprod_real(4, 4, 4, 8, a, b, c, nat.QT_SPLIT_BF16, None, 0, None),
      nat.qt_tprod_backward(4, 4, 4, 8, a, b, g, da, db, nat.QT_FP32, None, 0, None),
      nat.qt_tprod_batched(1, probs, nat.QT_FP32, None, 0, None),
      nat.qt_tprod(0, 4, 4, 8, a, b, c, nat.QT_FP32, None, 0, None))
"""


def test_injected_allocation_failure_returns_alloc():
    """QTPROD_FAULT=alloc makes the library's own workspace allocation
    (ws == NULL) fail: every one-shot product returns QT_ERR_ALLOC before any
    HIP call, while argument errors keep QT_ERR_INVALID_ARG (they are checked
    first).  Run in a child process: the variable is read once per process."""
    import subprocess
    import sys
    env = dict(os.environ, QTPROD_FAULT="alloc")
    out = subprocess.run([sys.executable, "-c", _FAULT_CHILD.format(root=ROOT)], env=env,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    got = [int(x) for x in out.stdout.split()]
    A = nat.QT_ERR_ALLOC
    assert got == [A, A, A, A, A, nat.QT_ERR_INVALID_ARG]
