"""Complex third-order tensors (a quaternion tensor whose second
Cayley-Dickson half is zero): the product uncouples into one complex matrix
product per frequency, C^(f) = A^(f) B^(f) (Algorithm 2.1 with the j-part of
Proposition 2.1 absent).  qt_tprod_complex is checked against the FP64
oracle on quaternion tensors with zero planes 2 and 3, and against a
complex block-circulant product formed directly in numpy."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import tprod_complex

from gpu_util import device, rel_err, sample_indices, to_dev, to_np

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "split_bf16": 5e-5, "split_fp16": 5e-5}


def _complex(rows, cols, p, seed):
    return synth.quat_tensor(rows, cols, p, seed=seed)[:2].copy()


def _as_quat(X):
    return np.concatenate([X, np.zeros_like(X)], axis=0)


def _bcirc_complex(A, B):
    """Definition of the T-product with complex faces: the block-circulant
    matrix of A's faces times the stacked faces of B."""
    a = A[0] + 1j * A[1]
    b = B[0] + 1j * B[1]
    p = a.shape[0]
    c = np.zeros((p, a.shape[1], b.shape[2]), complex)
    for k in range(p):
        for j in range(p):
            c[k] += a[(k - j) % p] @ b[j]
    return np.stack([c.real, c.imag])


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("m,n,s,p", [(300, 70, 90, 8), (64, 64, 64, 12), (33, 129, 5, 11), (1, 1, 1, 1),
                                     (257, 31, 65, 2), (20, 40, 30, 97)])
def test_complex_tprod(m, n, s, p, prec):
    A = _complex(m, n, p, seed=1500 + m)
    B = _complex(n, s, p, seed=1600 + s)
    C = tprod_complex(to_dev(A), to_dev(B), precision=prec)
    ref = oracle.tprod(_as_quat(A), _as_quat(B))
    assert np.abs(ref[2:]).max() == 0.0
    assert rel_err(to_np(C), ref[:2]) < TOLS[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_complex_large_tile_sampled(prec):
    """2 x 3 x 128 = 768 tiles of 256 x 128: the large complex tile (ragged in
    m and s), checked on sampled entries computed one by one."""
    m, n, s, p = 300, 40, 260, 128
    A = _complex(m, n, p, seed=1900)
    B = _complex(n, s, p, seed=1901)
    C = to_np(tprod_complex(to_dev(A), to_dev(B), precision=prec))
    k, i, j = sample_indices(p, m, s, 6, seed=1902, per_face=True)
    ref = oracle.tprod_entries(_as_quat(A), _as_quat(B), k, i, j)
    assert np.abs(ref[2:]).max() == 0.0
    got = C[:, k, i, j]
    err = float(np.sqrt(np.sum((got - ref[:2]) ** 2)) / np.sqrt(np.sum(ref[:2] ** 2)))
    assert err < TOLS[prec]


def test_complex_fp16_face_scales():
    """Split fp16 on complex tensors whose faces span 1e-3 .. 1e3: each
    frequency of A^ and of B^ gets its own power-of-two scale."""
    m, n, s, p = 70, 45, 60, 9
    rng = np.random.Generator(np.random.PCG64(1950))
    A = _complex(m, n, p, seed=1951) * (10.0 ** rng.uniform(-3, 3, p))[None, :, None, None]
    B = _complex(n, s, p, seed=1952) * (10.0 ** rng.uniform(-3, 3, p))[None, :, None, None]
    C = tprod_complex(to_dev(A), to_dev(B), precision="split_fp16")
    ref = oracle.tprod(_as_quat(A), _as_quat(B))[:2]
    err = rel_err(to_np(C), ref)
    print(f"complex split_fp16, face scales 1e-3..1e3: rel err {err:.3e}")
    assert err < TOLS["split_fp16"]


def test_complex_oracle_agrees_with_bcirc_definition():
    A = _complex(7, 5, 6, seed=1700)
    B = _complex(5, 4, 6, seed=1701)
    ref = oracle.tprod(_as_quat(A), _as_quat(B))[:2]
    assert rel_err(_bcirc_complex(A, B), ref) < 1e-13
    C = tprod_complex(to_dev(A), to_dev(B))
    assert rel_err(to_np(C), ref) < TOLS["fp32"]


def test_complex_out_and_workspace_reuse():
    m, n, s, p = 90, 50, 70, 16
    A = _complex(m, n, p, seed=1800)
    B = _complex(n, s, p, seed=1801)
    dev = device()
    out = torch.full((2, p, m, s), float("nan"), device=dev)
    ws = torch.empty(nat.qt_complex_workspace_size(m, n, s, p, nat.QT_SPLIT_BF16), dtype=torch.uint8, device=dev)
    ref = oracle.tprod(_as_quat(A), _as_quat(B))[:2]
    for prec in ("split_bf16", "fp32"):
        tprod_complex(to_dev(A), to_dev(B), precision=prec, out=out, ws=ws)
        assert rel_err(to_np(out), ref) < TOLS[prec]


def test_complex_rejects_quaternion_shape():
    A = torch.zeros((4, 2, 3, 3), device=device())
    with pytest.raises(ValueError):
        tprod_complex(A, A)
