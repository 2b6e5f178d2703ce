"""Fourier-domain-resident chains: (A * B) * C computed as three forward
transforms, two coupled products and one inverse transform, i.e. without the
inverse and forward transform of the intermediate A * B (bcirc(A * B) =
bcirc(A) bcirc(B), proof of Theorem 5.1).  For split-bf16 the FP32 product
is turned back into operand words in place by qt_split_words.  Checked
against the FP64 oracle applied twice."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import fourier_tprod, split_words, tube_fft

from gpu_util import device, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

# two chained products: about twice the single-product error
TOLS = {"fp32": 1e-5, "split_bf16": 5e-5}


def _fwd(X, prec):
    _, p, rows, cols = X.shape
    out = torch.empty((4, p, rows, nat.qt_fourier_ld(cols)), device=device())
    return tube_fft(to_dev(X), precision=prec, out=out)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("m,n,k,s,p", [(40, 24, 30, 20, 12), (130, 17, 66, 70, 5), (9, 3, 5, 7, 1)])
def test_chain_of_three(m, n, k, s, p, prec):
    A = synth.quat_tensor(m, n, p, seed=900)
    B = synth.quat_tensor(n, k, p, seed=901)
    C = synth.quat_tensor(k, s, p, seed=902)
    Ah, Bh, Ch = _fwd(A, prec), _fwd(B, prec), _fwd(C, prec)
    Xh = fourier_tprod(Ah, Bh, n, k, precision=prec)          # (A * B)^, FP32
    if prec == "split_bf16":
        split_words(Xh, cols=k)
    Dh = fourier_tprod(Xh, Ch, k, s, precision=prec)
    D = torch.empty((4, p, m, s), device=device())
    tube_fft(Dh, inverse=True, cols=s, out=D)
    ref = oracle.tprod(oracle.tprod(A, B), C)
    assert rel_err(to_np(D), ref) < TOLS[prec]


@pytest.mark.parametrize("p", [1, 8, 45])
def test_split_words_equals_split_transform(p):
    """qt_split_words on the FP32 transform gives exactly the words that the
    split-bf16 forward transform writes (same FFT arithmetic, same split)."""
    X = synth.quat_tensor(21, 30, p, seed=950 + p)
    F = _fwd(X, "fp32")
    split_words(F, cols=30)
    W = _fwd(X, "split_bf16")
    got = F[..., :30].contiguous().view(torch.int32).cpu().numpy()
    want = W[..., :30].contiguous().view(torch.int32).cpu().numpy()
    assert np.array_equal(got, want)
