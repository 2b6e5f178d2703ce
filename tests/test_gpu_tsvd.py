"""GPU quaternion t-SVD (qt_tsvd) against the FP64 oracle.

U and V are not unique, so they are checked by what they must satisfy:
A = U * S * V^H and U^H * U = I = V^H * V through the oracle's definitional
T-product.  S and sigma are unique (up to rounding) and are compared with the
oracle's entry by entry.

Tolerances.  The one-sided Jacobi stops rotating a pair of columns when their
cosine is below sqrt(2 max(m, n)) u (u the unit roundoff), so the factors are
orthonormal to about that level and A is reproduced to a few units of it:
FP32 is held to 2e-5 (relative Frobenius, and ||U^H * U - I||_F / sqrt(m)),
the singular values to 2e-5 of the largest; FP64 to 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import tsvd as ots
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import ops

from gpu_util import device, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-5, "fp64": 1e-12}


def _run(A64, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    _, p, m, n = A64.shape
    print(f"qt_tsvd {prec} m={m} n={n} p={p}", flush=True)
    U, S, V, sig = ops.tsvd(to_dev(A64, dt), precision=prec)
    torch.cuda.synchronize()
    return to_np(U), to_np(S), to_np(V), sig.double().cpu().numpy()


def _check(A64, prec, U, S, V, sig):
    tol = TOL[prec]
    _, p, m, n = A64.shape
    k = min(m, n)
    ref_U, ref_S, ref_V, ref_sig = ots.tsvd(A64)
    smax = max(float(ref_sig.max()), 1e-300)
    # unique parts
    assert np.abs(sig - ref_sig).max() <= tol * smax, f"sigma off by {np.abs(sig - ref_sig).max() / smax:.2e}"
    assert np.sqrt(oracle.qnorm2(S - ref_S)) <= tol * max(np.sqrt(oracle.qnorm2(ref_S)), 1e-300)
    off = S.copy()
    d = np.arange(k)
    off[:2][:, :, d, d] = 0
    assert np.abs(off).max() <= tol * smax, "S is not f-diagonal"
    # factors
    nA = np.sqrt(oracle.qnorm2(A64))
    R = oracle.tprod(oracle.tprod(U, S), oracle.tconjT(V))
    rec = np.sqrt(oracle.qnorm2(R - A64)) / max(nA, 1e-300)
    assert rec <= tol, f"reconstruction {rec:.2e}"
    for X, name in ((U, "U"), (V, "V")):
        r = X.shape[2]
        for G in (oracle.tprod(oracle.tconjT(X), X), oracle.tprod(X, oracle.tconjT(X))):
            e = np.sqrt(oracle.qnorm2(G - oracle.identity(r, p))) / np.sqrt(r)
            assert e <= tol, f"{name} not unitary: {e:.2e}"
    print(f"  sigma {np.abs(sig - ref_sig).max() / smax:.2e}  reconstruction {rec:.2e}", flush=True)


# ragged both ways, square, thin, p = 1, 2, odd, even, and Bluestein lengths
SHAPES = [(12, 7, 5), (7, 12, 6), (16, 16, 1), (9, 5, 2), (5, 9, 3), (1, 1, 4), (1, 6, 3), (6, 1, 7),
          (33, 20, 8), (20, 33, 11), (40, 40, 9), (64, 17, 13)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("m,n,p", SHAPES)
def test_tsvd_against_oracle(prec, m, n, p):
    A64 = synth.quat_tensor(m, n, p, seed=8000 + 97 * m + 13 * n + p)
    _check(A64, prec, *_run(A64, prec))


# Shapes with 2 min(m, n) >= 128 run the block sweeps (many workgroups per
# frequency pair, column blocks staged in LDS): ragged last blocks, an odd
# number of blocks (an idle slot in the schedule), wide and tall, p = 1 and
# p = 2 (quaternion pairs only) and odd p.
BLOCK_SHAPES = [(100, 70, 5), (70, 100, 4), (64, 64, 2), (90, 90, 1), (130, 67, 3)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("m,n,p", BLOCK_SHAPES)
def test_tsvd_block_sweeps_against_oracle(prec, m, n, p):
    A64 = synth.quat_tensor(m, n, p, seed=8050 + 97 * m + 13 * n + p)
    _check(A64, prec, *_run(A64, prec))


@pytest.mark.parametrize("prec,m,n,p", [("fp32", 1024, 64, 2), ("fp64", 400, 100, 3), ("fp32", 512, 512, 3)])
def test_tsvd_block_sweeps_small_blocks(prec, m, n, p):
    """Block sizes below eight units, where the staged columns are long: 4
    units per block (FP32, 1024 x 64: columns of 2048 entries) and 5 (FP64,
    400 x 100: a block size that is not a multiple of the eight waves); and
    FP32 512 x 512, eight units per block in a workgroup that has the CU's
    LDS to itself."""
    A64 = synth.quat_tensor(m, n, p, seed=8070 + m + n)
    _check(A64, prec, *_run(A64, prec))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tsvd_block_sweeps_rank_deficient(prec):
    X = synth.quat_tensor(96, 20, 3, seed=8110)
    Y = synth.quat_tensor(20, 80, 3, seed=8111)
    A64 = oracle.tprod(X, Y)            # chi_f(A) has rank <= 40 < 160
    U, S, V, sig = _run(A64, prec)
    _check(A64, prec, U, S, V, sig)
    assert np.all(sig[:, 20:] <= 10 * TOL[prec] * sig.max())


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tsvd_rank_deficient_and_zero(prec):
    X = synth.quat_tensor(14, 3, 6, seed=8100)
    Y = synth.quat_tensor(3, 10, 6, seed=8101)
    A64 = oracle.tprod(X, Y)            # chi_f(A) has rank <= 6 < 20
    U, S, V, sig = _run(A64, prec)
    _check(A64, prec, U, S, V, sig)
    assert np.all(sig[:, 3:] <= 10 * TOL[prec] * sig.max())
    Z = np.zeros((4, 5, 6, 4))
    U, S, V, sig = _run(Z, prec)
    assert np.all(sig == 0) and np.all(S == 0)
    for X in (U, V):
        r = X.shape[2]
        e = np.sqrt(oracle.qnorm2(oracle.tprod(oracle.tconjT(X), X) - oracle.identity(r, 5))) / np.sqrt(r)
        assert e <= TOL[prec]


def test_tsvd_real_and_complex_inputs():
    """Real input: the Fourier singular values are those of numpy's FFT faces
    (the real t-SVD); complex input: f and -f share those of both faces."""
    p, m, n = 6, 10, 7
    A = np.zeros((4, p, m, n))
    A[0] = synth.quat_tensor(m, n, p, seed=8200)[0]
    U, S, V, sig = _run(A, "fp32")
    want = np.linalg.svd(np.fft.fft(A[0], axis=0), compute_uv=False)
    np.testing.assert_allclose(sig, want, atol=2e-5 * want.max())
    _check(A, "fp32", U, S, V, sig)
    A = np.zeros((4, p, m, n))
    A[:2] = synth.quat_tensor(m, n, p, seed=8201)[:2]
    _check(A, "fp32", *_run(A, "fp32"))


def test_tsvd_scaled_inputs():
    """Tiny and huge magnitudes: each pair's matrix is scaled by a power of
    two before the Jacobi sweeps."""
    base = synth.quat_tensor(9, 6, 5, seed=8300)
    for sc in (1e-30, 1e25):
        A64 = base * sc
        U, S, V, sig = _run(A64, "fp32")
        _check(A64, "fp32", U, S, V, sig)


def test_tsvd_sizes_and_truncation():
    """256 x 192 x 16 (ragged, complex and quaternion pairs at full tile
    sizes): sigma against the oracle, reconstruction and the truncation error
    of the first r diagonal tubes, which must be (1/p) times the sum of the
    squared dropped Fourier singular values."""
    m, n, p = 256, 192, 16
    A64 = synth.quat_tensor(m, n, p, seed=8400)
    U, S, V, sig = _run(A64, "fp32")
    ref_sig = ots.tsvd(A64)[3]
    assert np.abs(sig - ref_sig).max() <= 2e-5 * ref_sig.max()
    nA2 = oracle.qnorm2(A64)
    for r in (n, 40):
        Sr = S.copy()
        Sr[:, :, r:, :] = 0
        Ar = oracle.tprod_faces(oracle.tprod_faces(U, Sr), oracle.tconjT(V))
        err2 = oracle.qnorm2(A64 - Ar)
        want = float(np.sum(ref_sig[:, r:] ** 2)) / p
        assert abs(err2 - want) <= 1e-4 * nA2, (r, err2, want)


def test_tsvd_argument_errors():
    dev = device()
    A = torch.zeros((4, 3, 5, 4), device=dev)
    U = torch.empty((4, 3, 5, 5), device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    # split precisions are not served
    st = nat.qt_tsvd(5, 4, 3, A.data_ptr(), U.data_ptr(), None, None, None, nat.QT_SPLIT_BF16, None, 0, stream)
    assert st == nat.QT_ERR_UNSUPPORTED
    # output overlapping the input
    st = nat.qt_tsvd(5, 4, 3, A.data_ptr(), A.data_ptr(), None, None, None, nat.QT_FP32, None, 0, stream)
    assert st == nat.QT_ERR_INVALID_ARG
    # beyond the size limits
    assert nat.qt_tsvd_workspace_size(600, 600, 3, nat.QT_FP32) == 0
    with pytest.raises(nat.QtError):
        ops.tsvd(torch.zeros((4, 2, 1100, 3), device=dev))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fourier_tsvd_stage_matches_qt_tsvd(prec):
    """qt_tube_fft + qt_fourier_tsvd + inverse transforms give bit for bit the
    U, V and sigma of qt_tsvd (same kernels on the same A^)."""
    dev = device()
    dt = torch.float64 if prec == "fp64" else torch.float32
    m, n, p = 21, 34, 7
    A64 = synth.quat_tensor(m, n, p, seed=8500)
    A = to_dev(A64, dt)
    U0, S0, V0, sig0 = ops.tsvd(A, precision=prec)
    P = nat.PRECISIONS[prec]
    lda, ldu, ldv = nat.qt_fourier_ld(n), nat.qt_fourier_ld(m), nat.qt_fourier_ld(n)
    Ah = torch.full((4, p, m, lda), float("nan"), dtype=dt, device=dev)
    Uh = torch.full((4, p, m, ldu), float("nan"), dtype=dt, device=dev)
    Vh = torch.full((4, p, n, ldv), float("nan"), dtype=dt, device=dev)
    sig = torch.empty((p, min(m, n)), dtype=dt, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    nat.check(nat.qt_tube_fft(m, n, p, A.data_ptr(), n, Ah.data_ptr(), lda, 0, P, stream), "fft")
    need = nat.qt_fourier_tsvd_workspace_size(m, n, p, P)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    st = nat.qt_fourier_tsvd(m, n, p, Ah.data_ptr(), lda, Uh.data_ptr(), ldu, Vh.data_ptr(), ldv, sig.data_ptr(),
                             P, ws.data_ptr(), need, stream)
    assert st == nat.QT_OK
    U = torch.empty((4, p, m, m), dtype=dt, device=dev)
    V = torch.empty((4, p, n, n), dtype=dt, device=dev)
    nat.check(nat.qt_tube_fft(m, m, p, Uh.data_ptr(), ldu, U.data_ptr(), m, 1, P, stream), "ifft U")
    nat.check(nat.qt_tube_fft(n, n, p, Vh.data_ptr(), ldv, V.data_ptr(), n, 1, P, stream), "ifft V")
    torch.cuda.synchronize()
    assert torch.equal(sig, sig0) and torch.equal(U, U0) and torch.equal(V, V0)
    assert nat.qt_fourier_tsvd(m, n, p, Ah.data_ptr(), lda, Uh.data_ptr(), ldu, Vh.data_ptr(), ldv, sig.data_ptr(),
                               P, ws.data_ptr(), need - 1, stream) == nat.QT_ERR_INVALID_ARG


def test_tsvd_full_workload_sampled():
    """The benchmarked workload: t-SVD of the 256x256x64 colour-video-like
    tensor (U[0,1), seed 2000).  sigma against the oracle's, S f-diagonal,
    and A = U * S * V^H on 256 sampled entries, with U * S formed from S's
    diagonal tubes and the entries of (U * S) * V^H computed one by one from
    the definition."""
    A64 = synth.config_inputs(2)[0]
    _, p, m, n = A64.shape
    U, S, V, sig = _run(A64, "fp32")
    ref_sig = ots.tsvd(A64)[3]
    assert np.abs(sig - ref_sig).max() <= 2e-5 * ref_sig.max()
    k = min(m, n)
    d = np.arange(k)
    off = S.copy()
    off[:2][:, :, d, d] = 0
    assert np.abs(off).max() <= 2e-5 * ref_sig.max()
    # U * S: column j of face f is sum_r U[:, f - r, :, j] * s_j[r] (S is f-diagonal, no j part)
    s_tube = S[0][:, d, d] + 1j * S[1][:, d, d]             # (p, k) complex diagonal tubes
    US = np.zeros((4, p, m, n))
    for f in range(p):
        for r in range(p):
            u = U[:, (f - r) % p][:, :, :k]                   # (4, m, k)
            c = s_tube[r]                                     # complex per column
            # (a + b i + c j + d k)(x + y i) for quaternion u and complex c
            a, b, cc, dd = u
            x, y = c.real, c.imag
            US[0, f, :, :k] += a * x - b * y
            US[1, f, :, :k] += a * y + b * x
            US[2, f, :, :k] += cc * x + dd * y
            US[3, f, :, :k] += dd * x - cc * y
    rng = np.random.Generator(np.random.PCG64(8600))
    kk, ii, jj = rng.integers(0, p, 256), rng.integers(0, m, 256), rng.integers(0, n, 256)
    got = oracle.tprod_entries(US, oracle.tconjT(V), kk, ii, jj)
    ref = A64[:, kk, ii, jj]
    err = float(np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2)))
    print(f"  full workload: sampled reconstruction {err:.2e}", flush=True)
    assert err <= 2e-5
