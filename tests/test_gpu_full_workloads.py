"""Full-size parity of the widened workloads in the launch configuration the
benchmark times (same inputs, same entry points, same tile choices): the
complex and real products and the Fourier-resident chain at 1024 x 1024 x
32, and the block-circulant mat-vec at 2048 x 2048 x 16.  Sampled output
entries are computed one by one by the oracle from the definition (for the
chain, from the oracle's FFT-form intermediate A * B)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import fourier_tprod, split_words, tprod_complex, tprod_real, tube_fft

from gpu_util import device, sample_indices, to_dev

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "split_bf16": 5e-5}


def _err(got, ref):
    return float(np.sqrt(np.sum((got - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))


def _embed(X, planes):
    return np.concatenate([X, np.zeros((4 - planes,) + X.shape[1:])])


@pytest.mark.parametrize("planes", [2, 1])
def test_complex_and_real_full_size(planes):
    A64, B64 = (x[:planes].copy() for x in synth.config_inputs(3)[:2])
    A, B = to_dev(A64), to_dev(B64)
    k, i, j = sample_indices(32, 1024, 1024, 4, seed=3300 + planes, per_face=True)
    ref = oracle.tprod_entries(_embed(A64, planes), _embed(B64, planes), k, i, j)
    assert np.abs(ref[planes:]).max() == 0.0
    for prec in ("fp32", "split_bf16"):
        if planes == 2:
            C = tprod_complex(A, B, prec).double().cpu().numpy()[:, k, i, j]
        else:
            C = tprod_real(A[0], B[0], prec).double().cpu().numpy()[None, k, i, j]
        err = _err(C, ref[:planes])
        print(f"{'complex' if planes == 2 else 'real'} {prec} sampled rel err {err:.3e}")
        assert err < TOLS[prec]


def test_chain_full_size():
    A64, B64 = synth.config_inputs(3)[:2]
    C64 = synth.quat_tensor(1024, 1024, 32, seed=3002)
    dev = device()
    ld = nat.qt_fourier_ld(1024)
    # X = A * B by the oracle's FFT form of Algorithm 5.1 (pinned against the
    # definition), then entries of X * C from the definition
    k, i, j = sample_indices(32, 1024, 1024, 4, seed=3400, per_face=True)
    X = oracle.tprod_fft(A64, B64)
    ref = oracle.tprod_entries(X, C64, k, i, j)
    del X
    for prec in ("fp32", "split_bf16"):
        Ah, Bh, Ch = (torch.empty((4, 32, 1024, ld), device=dev) for _ in range(3))
        tube_fft(to_dev(A64), precision=prec, out=Ah)
        tube_fft(to_dev(B64), precision=prec, out=Bh)
        tube_fft(to_dev(C64), precision=prec, out=Ch)
        Xh = fourier_tprod(Ah, Bh, 1024, 1024, precision=prec)
        if prec == "split_bf16":
            split_words(Xh, cols=1024)
        Dh = fourier_tprod(Xh, Ch, 1024, 1024, precision=prec, out=Ah)
        D = torch.empty((4, 32, 1024, 1024), device=dev)
        tube_fft(Dh, inverse=True, cols=1024, out=D)
        err = _err(D.double().cpu().numpy()[:, k, i, j], ref)
        print(f"chain {prec} sampled rel err {err:.3e}")
        assert err < TOLS[prec]
        del Ah, Bh, Ch, Xh, Dh, D


def test_matvec_full_size():
    m = n = 2048
    p = 16
    A64 = synth.quat_tensor(m, n, p, seed=6000)
    B64 = synth.quat_tensor(n, 1, p, seed=6001)
    dev = device()
    lda, ldb = nat.qt_fourier_ld(n), nat.qt_fourier_ld(1)
    k, i, j = sample_indices(p, m, 1, 16, seed=3500, per_face=True)
    ref = oracle.tprod_entries(A64, B64, k, i, j)
    for prec in ("fp32", "split_bf16"):
        Ah = torch.empty((4, p, m, lda), device=dev)
        Bh = torch.empty((4, p, n, ldb), device=dev)
        tube_fft(to_dev(A64), precision=prec, out=Ah)
        tube_fft(to_dev(B64), precision=prec, out=Bh)
        Ch = fourier_tprod(Ah, Bh, n, 1, precision=prec)
        C = torch.empty((4, p, m, 1), device=dev)
        tube_fft(Ch, inverse=True, cols=1, out=C)
        err = _err(C.double().cpu().numpy()[:, k, i, j], ref)
        print(f"matvec {prec} sampled rel err {err:.3e}")
        assert err < TOLS[prec]
