"""Torch-facing wrappers over the C-ABI: device memory, streams, autograd.

Torch supplies device buffers and the current HIP stream; every step of the
T-product runs in libqtprod's kernels.  Tensors are quaternion tensors in the
planar layout of the C-ABI: shape (4, p, rows, cols), contiguous, float32
(float64 for precision "fp64"), on a ROCm device.
"""
from __future__ import annotations

import torch

from . import _native as nat


def _prec(precision) -> int:
    if isinstance(precision, int):
        return precision
    try:
        return nat.PRECISIONS[precision]
    except KeyError:
        raise ValueError(f"unknown precision {precision!r}; use one of {list(nat.PRECISIONS)}")


def _dtype(prec: int):
    return torch.float64 if prec == nat.QT_FP64 else torch.float32


def _check_shape(x: torch.Tensor, name: str, planes: int = 4, shape=None,
                 min_last: int | None = None):
    """The library only sees pointers, so every size is checked here.
    shape: the full expected shape (None entries are free); min_last: lower
    bound of the last dimension (a row stride)."""
    if not isinstance(x, torch.Tensor) or x.dim() != 4 or x.shape[0] != planes:
        raise ValueError(f"{name} must be a tensor of shape ({planes}, p, rows, cols)")
    if shape is not None:
        if any(want is not None and got != want for got, want in zip(tuple(x.shape), shape)):
            want = tuple("*" if w is None else w for w in shape)
            raise ValueError(f"{name} has shape {tuple(x.shape)}, expected shape {want}")
    if min_last is not None and x.shape[3] < min_last:
        raise ValueError(f"{name} has shape {tuple(x.shape)}: its last dimension must be at least "
                         f"{min_last}")


def _check_storage(x: torch.Tensor, name: str, prec: int):
    if x.device.type != "cuda":
        raise ValueError(f"{name} must live on a ROCm device")
    if x.dtype != _dtype(prec):
        raise ValueError(f"{name} must be {_dtype(prec)} for this precision, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check_all(prec: int, *named):
    """Storage checks of several operands whose shapes were checked first."""
    for x, name in named:
        _check_storage(x, name, prec)


def _stream(dev) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def workspace(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer of at least nbytes (256-byte aligned by torch)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def tube_fft(X: torch.Tensor, inverse: bool = False, precision="fp32", cols=None,
             out: torch.Tensor | None = None) -> torch.Tensor:
    """Tube FFT of a quaternion tensor (block diagonalisation of bcirc(X)).

    X has shape (4, p, rows, ld); the first `cols` (default ld) columns are
    transformed.  `out` may have a different (padded) last dimension.
    """
    prec = _prec(precision)
    _check_shape(X, "X")
    _, p, rows, ldx = X.shape
    cols = ldx if cols is None else int(cols)
    if not 1 <= cols <= ldx:
        raise ValueError(f"cols must be in [1, {ldx}] for X of shape {tuple(X.shape)}")
    if out is not None:
        _check_shape(out, "out", shape=(4, p, rows, None), min_last=cols)
        _check_storage(out, "out", prec)
    _check_storage(X, "X", prec)
    if out is None:
        out = torch.empty_like(X)
    st = nat.qt_tube_fft(rows, cols, p, X.data_ptr(), ldx, out.data_ptr(), out.shape[3],
                         int(bool(inverse)), prec, _stream(X.device))
    nat.check(st, "qt_tube_fft")
    return out


def fourier_tprod(Ah: torch.Tensor, Bh: torch.Tensor, n: int, s: int, precision="fp32",
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """Coupled facewise product of Fourier-domain tensors (step 2 alone).

    Ah: (4, p, m, lda) holding n valid columns, Bh: (4, p, n, ldb) holding s
    valid columns; returns Ch (4, p, m, ldc) with s valid columns.
    """
    prec = _prec(precision)
    _check_shape(Ah, "Ah", min_last=n)
    _, p, m, lda = Ah.shape
    _check_shape(Bh, "Bh", shape=(4, p, n, None), min_last=s)
    ldb = Bh.shape[3]
    if out is not None:
        _check_shape(out, "out", shape=(4, p, m, None), min_last=s)
        _check_storage(out, "out", prec)
    _check_all(prec, (Ah, "Ah"), (Bh, "Bh"))
    if out is None:
        out = torch.empty((4, p, m, ldb), dtype=Ah.dtype, device=Ah.device)
    st = nat.qt_fourier_tprod(m, n, s, p, Ah.data_ptr(), lda, Bh.data_ptr(), ldb, out.data_ptr(),
                              out.shape[3], prec, _stream(Ah.device))
    nat.check(st, "qt_fourier_tprod")
    return out


def split_words(Xh: torch.Tensor, cols=None) -> torch.Tensor:
    """In place: Fourier-domain FP32 tensor (4, p, rows, ld) -> split-bf16
    operand words (the first `cols` columns, default ld); returns Xh."""
    _check_shape(Xh, "Xh")
    _, p, rows, ld = Xh.shape
    cols = ld if cols is None else int(cols)
    if not 1 <= cols <= ld:
        raise ValueError(f"cols must be in [1, {ld}] for Xh of shape {tuple(Xh.shape)}")
    _check_storage(Xh, "Xh", nat.QT_FP32)
    st = nat.qt_split_words(rows, cols, p, Xh.data_ptr(), ld, _stream(Xh.device))
    nat.check(st, "qt_split_words")
    return Xh


def tprod(A: torch.Tensor, B: torch.Tensor, precision="fp32", out: torch.Tensor | None = None,
          ws: torch.Tensor | None = None) -> torch.Tensor:
    """C = A * B (T-product of quaternion tensors) on the GPU."""
    prec = _prec(precision)
    _check_shape(A, "A")
    _, p, m, n = A.shape
    _check_shape(B, "B", shape=(4, p, n, None))
    s = B.shape[3]
    if out is not None:
        _check_shape(out, "out", shape=(4, p, m, s))
        _check_storage(out, "out", prec)
    _check_all(prec, (A, "A"), (B, "B"))
    if out is None:
        out = torch.empty((4, p, m, s), dtype=A.dtype, device=A.device)
    need = nat.qt_workspace_size(m, n, s, p, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, A.device)
    st = nat.qt_tprod(m, n, s, p, A.data_ptr(), B.data_ptr(), out.data_ptr(), prec,
                      ws.data_ptr(), ws.numel(), _stream(A.device))
    nat.check(st, "qt_tprod")
    return out


def tprod_complex(A: torch.Tensor, B: torch.Tensor, precision="fp32", out: torch.Tensor | None = None,
                  ws: torch.Tensor | None = None) -> torch.Tensor:
    """C = A * B for complex tensors of shape (2, p, rows, cols) = (Re, Im):
    one uncoupled complex product per frequency ("fp32" or "split_bf16")."""
    prec = _prec(precision)
    _check_shape(A, "A", planes=2)
    _, p, m, n = A.shape
    _check_shape(B, "B", planes=2, shape=(2, p, n, None))
    s = B.shape[3]
    if out is not None:
        _check_shape(out, "out", planes=2, shape=(2, p, m, s))
        _check_storage(out, "out", nat.QT_FP32)
    _check_all(nat.QT_FP32, (A, "A"), (B, "B"))
    if out is None:
        out = torch.empty((2, p, m, s), dtype=A.dtype, device=A.device)
    need = nat.qt_complex_workspace_size(m, n, s, p, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, A.device)
    st = nat.qt_tprod_complex(m, n, s, p, A.data_ptr(), B.data_ptr(), out.data_ptr(), prec,
                              ws.data_ptr(), ws.numel(), _stream(A.device))
    nat.check(st, "qt_tprod_complex")
    return out


def tprod_real(A: torch.Tensor, B: torch.Tensor, precision="fp32", out: torch.Tensor | None = None,
               ws: torch.Tensor | None = None) -> torch.Tensor:
    """C = A * B for real tensors of shape (p, rows, cols): frequencies
    0..p/2 only (Hermitian spectrum), one complex product each."""
    prec = _prec(precision)
    for x, name in ((A, "A"), (B, "B")):
        if not isinstance(x, torch.Tensor) or x.dim() != 3:
            raise ValueError(f"{name} must be a tensor of shape (p, rows, cols)")
    p, m, n = A.shape
    _check_shape(B.unsqueeze(0), "B", planes=1, shape=(1, p, n, None))
    s = B.shape[2]
    if out is not None:
        if not isinstance(out, torch.Tensor) or out.dim() != 3:
            raise ValueError("out must be a tensor of shape (p, m, s)")
        _check_shape(out.unsqueeze(0), "out", planes=1, shape=(1, p, m, s))
        _check_storage(out, "out", nat.QT_FP32)
    _check_all(nat.QT_FP32, (A, "A"), (B, "B"))
    if out is None:
        out = torch.empty((p, m, s), dtype=A.dtype, device=A.device)
    need = nat.qt_real_workspace_size(m, n, s, p, prec)
    if ws is None or ws.numel() < need:
        ws = workspace(need, A.device)
    st = nat.qt_tprod_real(m, n, s, p, A.data_ptr(), B.data_ptr(), out.data_ptr(), prec,
                           ws.data_ptr(), ws.numel(), _stream(A.device))
    nat.check(st, "qt_tprod_real")
    return out


def tprod_backward(A: torch.Tensor, B: torch.Tensor, G: torch.Tensor, precision="fp32",
                   need_dA: bool = True, need_dB: bool = True):
    """(dA, dB) = (G * B^H, A^H * G) on the GPU; None for a skipped one."""
    prec = _prec(precision)
    _check_shape(A, "A")
    _, p, m, n = A.shape
    _check_shape(B, "B", shape=(4, p, n, None))
    s = B.shape[3]
    _check_shape(G, "G", shape=(4, p, m, s))
    _check_all(prec, (A, "A"), (B, "B"), (G, "G"))
    dA = torch.empty_like(A) if need_dA else None
    dB = torch.empty_like(B) if need_dB else None
    need = nat.qt_backward_workspace_size(m, n, s, p, prec)
    ws = workspace(need, A.device)
    st = nat.qt_tprod_backward(m, n, s, p, A.data_ptr(), B.data_ptr(), G.data_ptr(),
                               dA.data_ptr() if dA is not None else None,
                               dB.data_ptr() if dB is not None else None,
                               prec, ws.data_ptr(), ws.numel(), _stream(A.device))
    nat.check(st, "qt_tprod_backward")
    return dA, dB


def _check_problem(A, B, C, prec):
    """One problem of a batch: A m x n x p, B n x s x p, C m x s x p."""
    _check_shape(A, "A")
    _, p, m, n = A.shape
    _check_shape(B, "B", shape=(4, p, n, None))
    _check_shape(C, "C", shape=(4, p, m, B.shape[3]))
    _check_all(prec, (A, "A"), (B, "B"), (C, "C"))


def tprod_batched(As, Bs, precision="fp32", outs=None):
    """[A_i * B_i] for lists of tensors in one call of the batched path
    (tube FFTs per distinct p, one persistent product launch per tile shape)."""
    prec = _prec(precision)
    if len(As) != len(Bs) or not As:
        raise ValueError("need equally many A and B tensors (at least one)")
    items = []
    if outs is not None and len(outs) != len(As):
        raise ValueError("need one output tensor per problem")
    for A, B in zip(As, Bs):
        _check_shape(A, "A")
        _check_shape(B, "B", shape=(4, A.shape[1], A.shape[3], None))
    if outs is None:
        outs = []
        for A, B in zip(As, Bs):
            outs.append(torch.empty((4, A.shape[1], A.shape[2], B.shape[3]), dtype=A.dtype,
                                    device=A.device))
    for A, B, C in zip(As, Bs, outs):
        _check_problem(A, B, C, prec)
        items.append((A.shape[2], A.shape[3], B.shape[3], A.shape[1], A.data_ptr(), B.data_ptr(),
                      C.data_ptr()))
    probs = nat.make_problems(items)
    need = nat.qt_batched_workspace_size(len(items), probs, prec)
    ws = workspace(need, As[0].device)
    st = nat.qt_tprod_batched(len(items), probs, prec, ws.data_ptr(), ws.numel(),
                              _stream(As[0].device))
    nat.check(st, "qt_tprod_batched")
    return outs


class BatchedPlan:
    """A captured batch: C_i = A_i * B_i for fixed tensors, replayed with one
    hipGraphLaunch per call.  Keeps the tensors and the workspace alive."""

    def __init__(self, As, Bs, precision="fp32", outs=None):
        prec = _prec(precision)
        if len(As) != len(Bs) or not As:
            raise ValueError("need equally many A and B tensors (at least one)")
        if outs is not None and len(outs) != len(As):
            raise ValueError("need one output tensor per problem")
        for A, B in zip(As, Bs):
            _check_shape(A, "A")
            _check_shape(B, "B", shape=(4, A.shape[1], A.shape[3], None))
        if outs is None:
            outs = [torch.empty((4, A.shape[1], A.shape[2], B.shape[3]), dtype=A.dtype,
                                device=A.device) for A, B in zip(As, Bs)]
        items = []
        for A, B, C in zip(As, Bs, outs):
            _check_problem(A, B, C, prec)
            items.append((A.shape[2], A.shape[3], B.shape[3], A.shape[1], A.data_ptr(),
                          B.data_ptr(), C.data_ptr()))
        self._keep = (list(As), list(Bs))
        self.outs = outs
        probs = nat.make_problems(items)
        need = nat.qt_batched_workspace_size(len(items), probs, prec)
        self.ws = workspace(need, As[0].device)
        self.device = As[0].device
        st, self.handle = nat.qt_batched_plan_create(len(items), probs, prec, self.ws.data_ptr(),
                                                     self.ws.numel(), _stream(self.device))
        nat.check(st, "qt_batched_plan_create")

    def launch(self):
        nat.check(nat.qt_batched_plan_launch(self.handle, _stream(self.device)),
                  "qt_batched_plan_launch")
        return self.outs

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.current_stream(self.device).synchronize()
            nat.check(nat.qt_batched_plan_destroy(self.handle), "qt_batched_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(precision="fp32", device=None):
    """Run the device autotuner (tile cost model, FFT radix orders) now."""
    dev = device or torch.device("cuda", torch.cuda.current_device())
    nat.check(nat.qt_autotune(_prec(precision), _stream(dev)), "qt_autotune")


def tsvd(A: torch.Tensor, precision="fp32", ws: torch.Tensor | None = None):
    """Quaternion t-SVD A = U * S * V^H on the GPU.

    A: (4, p, m, n).  Returns (U (4, p, m, m), S (4, p, m, n), V (4, p, n, n),
    sigma (p, min(m, n))), sigma[f, i] being entry (i, i) of S1^[f].
    precision: "fp32" or "fp64"."""
    prec = _prec(precision)
    _check_shape(A, "A")
    _, p, m, n = A.shape
    _check_storage(A, "A", prec)
    opts = dict(dtype=A.dtype, device=A.device)
    U = torch.empty((4, p, m, m), **opts)
    S = torch.empty((4, p, m, n), **opts)
    V = torch.empty((4, p, n, n), **opts)
    sigma = torch.empty((p, min(m, n)), **opts)
    need = nat.qt_tsvd_workspace_size(m, n, p, prec)
    if need == 0:     # split precisions, or sizes beyond the limits
        nat.check(nat.QT_ERR_UNSUPPORTED, "qt_tsvd")
    if ws is None or ws.numel() < need:
        ws = workspace(need, A.device)
    st = nat.qt_tsvd(m, n, p, A.data_ptr(), U.data_ptr(), S.data_ptr(), V.data_ptr(), sigma.data_ptr(),
                     prec, ws.data_ptr(), ws.numel(), _stream(A.device))
    nat.check(st, "qt_tsvd")
    return U, S, V, sigma


class QTProd(torch.autograd.Function):
    """C = A * B with the hand-written Fourier-domain backward.

    Gradients are plain real gradients of the four component planes:
    dL/dA = G * B^H, dL/dB = A^H * G for G = dL/dC.
    """

    @staticmethod
    def forward(ctx, A, B, precision="fp32"):
        ctx.precision = precision
        A, B = A.contiguous(), B.contiguous()
        ctx.save_for_backward(A, B)          # the contiguous tensors the backward needs
        return tprod(A, B, precision)

    @staticmethod
    def backward(ctx, G):
        A, B = ctx.saved_tensors
        dA, dB = tprod_backward(A, B, G.contiguous(), ctx.precision,
                                need_dA=ctx.needs_input_grad[0], need_dB=ctx.needs_input_grad[1])
        return dA, dB, None


def qtprod(A, B, precision="fp32"):
    """Differentiable T-product (autograd through QTProd)."""
    return QTProd.apply(A, B, precision)
