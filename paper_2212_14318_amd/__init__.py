"""MI355X-native fast T-product of third-order quaternion tensors.

C = A * B for A (m x n x p) and B (n x s x p) quaternion tensors, computed as
tube FFT -> coupled facewise complex products -> inverse tube FFT in
hand-written HIP kernels for gfx950 (libqtprod.so, C-ABI in include/qtprod.h).

Quaternion tensors are torch tensors of shape (4, p, rows, cols): the planes
are the real components (a, b, c, d) of a + b i + c j + d k, i.e. the
Cayley-Dickson parts X1 = a + b i and X2 = c + d i.

    from paper_2212_14318_amd import tprod, qtprod
    C = tprod(A, B, precision="fp32")     # or "split_bf16", "fp64"
    C = qtprod(A, B)                      # differentiable (autograd.Function)
    U, S, V, sigma = tsvd(A)              # quaternion t-SVD, A = U * S * V^H
"""
from .ops import (BatchedPlan, QTProd, autotune, fourier_tprod, qtprod, split_words, tprod,  # noqa: F401
                  tprod_backward, tprod_batched, tprod_complex, tprod_real, tsvd, tube_fft)
from ._native import PRECISIONS, QtError  # noqa: F401

__all__ = ["tprod", "tprod_complex", "tprod_real", "tube_fft", "fourier_tprod", "split_words", "BatchedPlan", "autotune", "tprod_backward", "tprod_batched", "tsvd", "qtprod", "QTProd", "PRECISIONS", "QtError"]
