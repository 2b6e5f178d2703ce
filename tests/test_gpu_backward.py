"""GPU parity of the hand-written backward (qt_tprod_backward, QTProd).

dA = G * B^H and dB = A^H * G are compared with the oracle's adjoints
(definitional T-products with the tensor conjugate transpose), and on the
full-size differentiation workload with FP64 central differences of
L = 1/2 ||A * B - T||_F^2 on a 16 x 4 x 10 slice of A and of B."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.quaternion import qmul
from paper_2212_14318_amd import qtprod, tprod, tprod_backward

from gpu_util import rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "split_bf16": 5e-5, "split_fp16": 5e-5, "fp64": 1e-13}
DT = {"fp32": torch.float32, "split_bf16": torch.float32, "split_fp16": torch.float32, "fp64": torch.float64}


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16", "fp64"])
@pytest.mark.parametrize("m,n,s,p", [(8, 8, 8, 8), (37, 21, 50, 5), (150, 40, 130, 12),
                                     (1, 1, 1, 1), (3, 70, 2, 7)])
def test_backward_matches_oracle(prec, m, n, s, p):
    A = synth.quat_tensor(m, n, p, seed=10 + m + p)
    B = synth.quat_tensor(n, s, p, seed=20 + s + p)
    G = synth.quat_tensor(m, s, p, seed=30 + n + p)
    dA, dB = tprod_backward(to_dev(A, DT[prec]), to_dev(B, DT[prec]), to_dev(G, DT[prec]), prec)
    rA, rB = oracle.adjoints(A, B, G)
    ea, eb = rel_err(to_np(dA), rA), rel_err(to_np(dB), rB)
    print(f"{prec} {m}x{n}x{s} p={p}: dA {ea:.3e} dB {eb:.3e}")
    assert ea <= TOLS[prec] and eb <= TOLS[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_fp16"])
def test_backward_one_sided(prec):
    m, n, s, p = 40, 24, 33, 6
    A = synth.quat_tensor(m, n, p, seed=41)
    B = synth.quat_tensor(n, s, p, seed=42)
    G = synth.quat_tensor(m, s, p, seed=43)
    rA, rB = oracle.adjoints(A, B, G)
    dA, dB = tprod_backward(to_dev(A), to_dev(B), to_dev(G), prec, need_dB=False)
    assert dB is None and rel_err(to_np(dA), rA) <= TOLS[prec]
    dA, dB = tprod_backward(to_dev(A), to_dev(B), to_dev(G), prec, need_dA=False)
    assert dA is None and rel_err(to_np(dB), rB) <= TOLS[prec]


def test_adjoint_dot_identity_gpu():
    """<A * B, Z> = <A, Z * B^H> = <B, A^H * Z> with GPU products."""
    m, n, s, p = 64, 48, 80, 10
    A = synth.quat_tensor(m, n, p, seed=51)
    B = synth.quat_tensor(n, s, p, seed=52)
    Z = synth.quat_tensor(m, s, p, seed=53)
    Ad, Bd, Zd = to_dev(A, torch.float64), to_dev(B, torch.float64), to_dev(Z, torch.float64)
    C = tprod(Ad, Bd, precision="fp64")
    dA, dB = tprod_backward(Ad, Bd, Zd, "fp64")
    lhs = float((C * Zd).sum())
    assert abs(lhs - float((Ad * dA).sum())) <= 1e-11 * abs(lhs)
    assert abs(lhs - float((Bd * dB).sum())) <= 1e-11 * abs(lhs)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_autograd_function(prec):
    m, n, s, p = 60, 20, 44, 9
    A64 = synth.quat_tensor(m, n, p, seed=61)
    B64 = synth.quat_tensor(n, s, p, seed=62)
    T64 = synth.quat_tensor(m, s, p, seed=63)
    A = to_dev(A64).requires_grad_(True)
    B = to_dev(B64).requires_grad_(True)
    T = to_dev(T64)
    loss = 0.5 * ((qtprod(A, B, prec) - T) ** 2).sum()
    loss.backward()
    G = oracle.tprod(A64, B64) - T64
    rA, rB = oracle.adjoints(A64, B64, G)
    assert rel_err(to_np(A.grad), rA) <= 5e-5
    assert rel_err(to_np(B.grad), rB) <= 5e-5


def _fd_slice_grad_A(A, B, T, rows, cols, faces, h=1e-3):
    """Central differences of L = 1/2 ||A * B - T||^2 w.r.t. A[c, k, i, j].

    Only row i of A * B depends on A[:, :, i, :], and the product is linear in
    A, so L(A +- h E) is evaluated exactly from row i of the FP64 residual and
    the change h * (e_c . B[(k - k0) mod p][j, :]) of that row (definition of
    the T-product, Section 2.4)."""
    p = A.shape[1]
    R = oracle.tprod_rows(A, B, rows) - T[:, :, rows, :]          # (4, p, len(rows), s)
    out = np.zeros((4, len(faces), len(rows), len(cols)))
    for ri, i in enumerate(rows):
        Ri = R[:, :, ri, :]                                        # (4, p, s)
        for ci, j in enumerate(cols):
            for fi, k0 in enumerate(faces):
                Bj = B[:, (np.arange(p) - k0) % p, j, :]           # (4, p, s): face k uses B[k - k0]
                for c in range(4):
                    e = np.zeros((4, 1, 1)); e[c] = 1.0
                    delta = qmul(e, Bj)                             # change of row i per unit h
                    lp = 0.5 * np.sum((Ri + h * delta) ** 2)
                    lm = 0.5 * np.sum((Ri - h * delta) ** 2)
                    out[c, fi, ri, ci] = (lp - lm) / (2 * h)
    return out


def _fd_slice_grad_B(A, B, T, rows, cols, faces, h=1e-3):
    """Central differences w.r.t. B[c, k, l, j]: only column j of A * B moves,
    by h * (A[(k - k0) mod p][:, l] . e_c) on every face k."""
    p = A.shape[1]
    out = np.zeros((4, len(faces), len(rows), len(cols)))
    R = oracle.tprod_cols(A, B, cols) - T[:, :, :, cols]          # (4, p, m, len(cols))
    for ri, l in enumerate(rows):
        for ci, j in enumerate(cols):
            Rj = R[:, :, :, ci]                                    # (4, p, m)
            for fi, k0 in enumerate(faces):
                # A[:, (k - k0) mod p, :, l] comes out as (p, 4, m): move to (4, p, m)
                Al = np.moveaxis(A[:, (np.arange(p) - k0) % p, :, l], 0, 1)
                for c in range(4):
                    e = np.zeros((4, 1, 1)); e[c] = 1.0
                    delta = qmul(Al, e)
                    lp = 0.5 * np.sum((Rj + h * delta) ** 2)
                    lm = 0.5 * np.sum((Rj - h * delta) ** 2)
                    out[c, fi, ri, ci] = (lp - lm) / (2 * h)
    return out


def test_c5_full_size_fd_and_oracle():
    A, B, T = synth.config_inputs(5)
    _, p, m, n = A.shape
    s = B.shape[3]
    Ad, Bd, Td = to_dev(A), to_dev(B), to_dev(T)
    C = tprod(Ad, Bd)
    G = (C - Td).contiguous()
    dA, dB = tprod_backward(Ad, Bd, G)
    dA, dB = to_np(dA), to_np(dB)
    # (1) FP64 finite differences on the 16 x 4 x 10 slice of A and of B
    rows, cols, faces = list(range(16)), list(range(4)), list(range(10))
    print("c5: FD of dA on the slice", flush=True)
    fdA = _fd_slice_grad_A(A, B, T, rows, cols, faces)
    gotA = dA[:, :10, :16, :4]
    eA = rel_err(gotA, fdA)
    print("c5: FD of dB on the slice", flush=True)
    fdB = _fd_slice_grad_B(A, B, T, rows, cols, faces)
    gotB = dB[:, :10, :16, :4]
    eB = rel_err(gotB, fdB)
    print(f"c5 FD slice: dA {eA:.3e}  dB {eB:.3e}")
    assert eA <= 1e-5 and eB <= 1e-5
    # (2) oracle adjoints on sampled entries of dA = G * B^H and dB = A^H * G
    G64 = to_np(G)
    rng = np.random.Generator(np.random.PCG64(5100))
    k = rng.integers(0, p, 300); i = rng.integers(0, m, 300); j = rng.integers(0, n, 300)
    refA = oracle.tprod_entries(G64, oracle.tconjT(B), k, i, j)
    ea = np.sqrt(np.sum((dA[:, k, i, j] - refA) ** 2) / np.sum(refA ** 2))
    k2 = rng.integers(0, p, 300); i2 = rng.integers(0, n, 300); j2 = rng.integers(0, s, 300)
    refB = oracle.tprod_entries(oracle.tconjT(A), G64, k2, i2, j2)
    eb = np.sqrt(np.sum((dB[:, k2, i2, j2] - refB) ** 2) / np.sum(refB ** 2))
    print(f"c5 oracle adjoint sampled: dA {ea:.3e}  dB {eb:.3e}")
    assert ea <= 1e-5 and eb <= 1e-5
