"""Real third-order tensors: the T-product of Algorithm 2.1 on real input.
The tube DFT of a real tensor is Hermitian, so qt_tprod_real transforms,
multiplies and inverts only frequencies 0..p/2.  Checked against the FP64
oracle on quaternion tensors whose planes 1..3 are zero, and the oracle
against the real block-circulant product written out in numpy."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import tprod_complex, tprod_real

from gpu_util import device, rel_err, sample_indices, to_dev, to_np

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "split_bf16": 5e-5, "split_fp16": 5e-5}


def _real(rows, cols, p, seed):
    return synth.quat_tensor(rows, cols, p, seed=seed)[0].copy()


def _as_quat(X):
    Q = np.zeros((4,) + X.shape)
    Q[0] = X
    return Q


def _bcirc_real(A, B):
    p = A.shape[0]
    C = np.zeros((p, A.shape[1], B.shape[2]))
    for k in range(p):
        for j in range(p):
            C[k] += A[(k - j) % p] @ B[j]
    return C


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("m,n,s,p", [(300, 70, 90, 8), (64, 64, 64, 12), (33, 129, 5, 11), (1, 1, 1, 1),
                                     (257, 31, 65, 2), (20, 40, 30, 97), (50, 20, 70, 3), (40, 33, 20, 128),
                                     (24, 17, 9, 200)])
def test_real_tprod(m, n, s, p, prec):
    A = _real(m, n, p, seed=2500 + m)
    B = _real(n, s, p, seed=2600 + s)
    C = tprod_real(to_dev(A), to_dev(B), precision=prec)
    ref = oracle.tprod(_as_quat(A), _as_quat(B))
    assert np.abs(ref[1:]).max() == 0.0
    assert rel_err(to_np(C), ref[0]) < TOLS[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_real_large_tile_sampled(prec):
    """p = 256 keeps 129 frequencies: 2 x 3 x 129 tiles of 256 x 128 (ragged in
    m and s), checked on sampled entries computed one by one."""
    m, n, s, p = 300, 20, 260, 256
    A = _real(m, n, p, seed=3200)
    B = _real(n, s, p, seed=3201)
    C = to_np(tprod_real(to_dev(A), to_dev(B), precision=prec))
    k, i, j = sample_indices(p, m, s, 4, seed=3202, per_face=True)
    ref = oracle.tprod_entries(_as_quat(A), _as_quat(B), k, i, j)
    assert np.abs(ref[1:]).max() == 0.0
    got = C[k, i, j]
    err = float(np.sqrt(np.sum((got - ref[0]) ** 2)) / np.sqrt(np.sum(ref[0] ** 2)))
    assert err < TOLS[prec]


def test_real_oracle_agrees_with_bcirc_definition():
    A = _real(7, 5, 6, seed=2700)
    B = _real(5, 4, 6, seed=2701)
    ref = oracle.tprod(_as_quat(A), _as_quat(B))[0]
    assert rel_err(_bcirc_real(A, B), ref) < 1e-13
    assert rel_err(to_np(tprod_real(to_dev(A), to_dev(B))), ref) < TOLS["fp32"]


@pytest.mark.parametrize("p", [5, 16, 45])
def test_real_matches_complex_path(p):
    """The half-spectrum path and the full complex path (zero imaginary
    planes) compute the same product."""
    A = _real(70, 40, p, seed=2800 + p)
    B = _real(40, 66, p, seed=2900 + p)
    Cr = to_np(tprod_real(to_dev(A), to_dev(B)))
    Ac = np.stack([A, np.zeros_like(A)])
    Bc = np.stack([B, np.zeros_like(B)])
    Cc = to_np(tprod_complex(to_dev(Ac), to_dev(Bc)))
    assert rel_err(Cr, Cc[0]) < 2e-6
    assert np.abs(Cc[1]).max() <= 1e-5 * np.abs(Cc[0]).max()


def test_real_out_and_workspace_reuse():
    m, n, s, p = 90, 50, 70, 16
    A = _real(m, n, p, seed=3100)
    B = _real(n, s, p, seed=3101)
    dev = device()
    out = torch.full((p, m, s), float("nan"), device=dev)
    ws = torch.empty(nat.qt_real_workspace_size(m, n, s, p, nat.QT_SPLIT_BF16), dtype=torch.uint8, device=dev)
    ref = oracle.tprod(_as_quat(A), _as_quat(B))[0]
    for prec in ("split_bf16", "fp32"):
        tprod_real(to_dev(A), to_dev(B), precision=prec, out=out, ws=ws)
        assert rel_err(to_np(out), ref) < TOLS[prec]


def test_real_rejects_bad_shapes():
    dev = device()
    A = torch.zeros((4, 3, 3), device=dev)
    with pytest.raises(ValueError):
        tprod_real(A, torch.zeros((4, 2, 3), device=dev))
    with pytest.raises(ValueError):
        tprod_real(torch.zeros((2, 4, 3, 3), device=dev), A)
