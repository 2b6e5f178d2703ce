"""Narrow products (s <= 4 columns): a block-circulant quaternion matrix
times a few tube vectors, which run the FP32 VALU mat-vec kernel in every
float precision.  Parity against the FP64 oracle; the k tails cross the
kernel's 256-deep k tiles."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import fourier_tprod, tprod, tube_fft

from gpu_util import device, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

# the narrow kernel computes in FP32 on FP32 operands (split-bf16: on the
# decoded words hi + lo, ~16 significant bits)
TOLS = {"fp32": 1e-5, "split_bf16": 5e-5, "split_fp16": 1e-5}


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("m,n,s,p", [(37, 300, 1, 7), (20, 513, 2, 12), (65, 64, 3, 32), (16, 257, 4, 5),
                                     (1, 1, 1, 1), (3, 2, 4, 2)])
def test_narrow_tprod(m, n, s, p, prec):
    A = synth.quat_tensor(m, n, p, seed=1200 + n)
    B = synth.quat_tensor(n, s, p, seed=1300 + n)
    C = tprod(to_dev(A), to_dev(B), precision=prec)
    assert rel_err(to_np(C), oracle.tprod(A, B)) < TOLS[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_narrow_staged_path(prec):
    """qt_fourier_tprod with s = 1 on transformed operands (split words for
    split-bf16), padded row strides."""
    m, n, s, p = 50, 300, 1, 8
    A = synth.quat_tensor(m, n, p, seed=1400)
    B = synth.quat_tensor(n, s, p, seed=1401)
    dev = device()
    Ah = torch.empty((4, p, m, nat.qt_fourier_ld(n)), device=dev)
    Bh = torch.empty((4, p, n, nat.qt_fourier_ld(s)), device=dev)
    tube_fft(to_dev(A), precision=prec, out=Ah)
    tube_fft(to_dev(B), precision=prec, out=Bh)
    Ch = fourier_tprod(Ah, Bh, n, s, precision=prec)
    C = torch.empty((4, p, m, s), device=dev)
    tube_fft(Ch, inverse=True, cols=s, out=C)
    assert rel_err(to_np(C), oracle.tprod(A, B)) < TOLS[prec]


@pytest.mark.parametrize("p", [5, 16, 97])
def test_circular_quaternion_convolution(p):
    """m = n = s = 1: the T-product of two tubes is their circular convolution
    with quaternion (Hamilton) products, c_k = sum_r a_{k - r} b_r."""
    a = synth.quat_tensor(1, 1, p, seed=1500 + p)
    b = synth.quat_tensor(1, 1, p, seed=1600 + p)
    got = to_np(tprod(to_dev(a), to_dev(b)))
    want = np.zeros_like(a)
    for k in range(p):
        for r in range(p):
            want[:, k, 0, 0] += oracle.qmul(a[:, (k - r) % p, 0, 0], b[:, r, 0, 0])
    assert rel_err(got, want) < 1e-5
