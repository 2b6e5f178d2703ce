"""GPU parity of the forward T-product (qt_tprod, qt_tube_fft) against the
FP64 oracle.  Tolerances: relative Frobenius error <= 1e-5 for the FP32 path
and <= 1e-13 for the FP64 path (the paper observes ~1e-16 for the fast
algorithm in FP64; 1e-13 leaves room for the accumulation order)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import fourier_tprod, tprod, tube_fft

from gpu_util import device, rel_err, sample_indices, sampled_rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_TOL = 1e-13
# split bf16 (hi + lo, three products): the stated gate is 2e-3; the expected
# error is ~4e-6 (dropped lo*lo term ~2^-16 relative plus FP32 rounding), so
# the tests hold it to 5e-5, which a plain (unsplit) bf16 product (~2e-3)
# cannot meet.
SPLIT_GATE = 2e-3
SPLIT_GUARD = 5e-5
TOLS = {"fp32": FP32_TOL, "split_bf16": SPLIT_GUARD, "split_fp16": SPLIT_GUARD}
PRECS = ["fp32", "split_bf16", "split_fp16"]


# ------------------------------------------------------------------ tube FFT
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 30, 32, 45, 49, 64, 100, 125, 128])
def test_tube_fft_matches_numpy(p):
    rows, cols = 13, 37
    X = synth.quat_tensor(rows, cols, p, seed=100 + p)
    Xd = to_dev(X)
    H = to_np(tube_fft(Xd))
    want1 = np.fft.fft(X[0] + 1j * X[1], axis=0)
    want2 = np.fft.fft(X[2] + 1j * X[3], axis=0)
    want = np.stack([want1.real, want1.imag, want2.real, want2.imag])
    assert rel_err(H, want) < 2e-6
    back = to_np(tube_fft(to_dev(want), inverse=True))
    assert rel_err(back, X) < 2e-6


@pytest.mark.parametrize("rows,cols,p", [(70, 45, 32), (33, 101, 45), (300, 7, 16), (64, 64, 12), (50, 257, 64)])
def test_tube_fft_unaligned_faces(rows, cols, p):
    """Faces whose size is not a multiple of 32 reals (each face starts at a
    different offset within a cache line), multi-block: forward from the
    dense layout into padded Fourier rows (FP32 and split words), inverse from
    the padded rows back to the dense layout.  64 x 64 is the aligned control.
    The caller's padding columns keep their contents (only the library's own
    workspaces get their padding written)."""
    X = synth.quat_tensor(rows, cols, p, seed=170 + p)
    dev = device()
    F = torch.full((4, p, rows, nat.qt_fourier_ld(cols)), 7.0, device=dev)
    tube_fft(to_dev(X), out=F)
    assert bool((F[..., cols:] == 7.0).all())
    w1 = np.fft.fft(X[0] + 1j * X[1], axis=0)
    w2 = np.fft.fft(X[2] + 1j * X[3], axis=0)
    want = np.stack([w1.real, w1.imag, w2.real, w2.imag])
    assert rel_err(to_np(F[..., :cols]), want) < 2e-6
    back = torch.empty((4, p, rows, cols), device=dev)
    tube_fft(F, inverse=True, cols=cols, out=back)
    assert rel_err(to_np(back), X) < 2e-6
    W = torch.full_like(F, 7.0)
    tube_fft(to_dev(X), precision="split_bf16", out=W)
    assert bool((W[..., cols:] == 7.0).all())
    hi, lo = _unpack_split_words(W[..., :cols])
    assert rel_err(hi + lo, want) < 2e-5


def _unpack_split_words(t):
    """(hi | lo << 16) bf16 words -> hi + lo as float64."""
    w = t.contiguous().view(torch.int32).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    hi = ((w & 0xFFFF) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    lo = ((w >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return hi, lo


@pytest.mark.parametrize("p", [1, 7, 32, 64])
def test_tube_fft_split_words(p):
    """Forward transform in the split-bf16 operand format: each word holds
    hi = rn_bf16(x) and lo = rn_bf16(x - hi); hi + lo keeps ~16 bits."""
    rows, cols = 9, 33
    X = synth.quat_tensor(rows, cols, p, seed=150 + p)
    H = tube_fft(to_dev(X), precision="split_bf16")
    hi, lo = _unpack_split_words(H)
    w1 = np.fft.fft(X[0] + 1j * X[1], axis=0)
    w2 = np.fft.fft(X[2] + 1j * X[3], axis=0)
    want = np.stack([w1.real, w1.imag, w2.real, w2.imag])
    assert rel_err(hi + lo, want) < 2e-5
    assert rel_err(hi, want) < 1e-2          # hi alone is only a bf16 rounding
    assert np.all(np.abs(lo) <= np.abs(hi) * 2.0 ** -8 + 1e-30)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("m,n,s,p", [(300, 50, 150, 12), (250, 33, 65, 8), (130, 17, 70, 5),
                                     (129, 16, 65, 3), (64, 1, 64, 2)])
def test_staged_path_ragged(m, n, s, p, prec):
    """The three stages called one by one (qt_tube_fft, qt_fourier_tprod,
    inverse qt_tube_fft), with padded Fourier row strides.  qt_fourier_tprod
    always runs the 128 x 64 tile (for split-bf16 the two-plane-group
    kernel), so these shapes pin its edge tiles, k tails and padding."""
    A = synth.quat_tensor(m, n, p, seed=700 + m)
    B = synth.quat_tensor(n, s, p, seed=800 + s)
    lda, ldb = nat.qt_fourier_ld(n), nat.qt_fourier_ld(s)
    dev = device()
    Ah = torch.full((4, p, m, lda), float("nan"), device=dev)
    Bh = torch.full((4, p, n, ldb), float("nan"), device=dev)
    tube_fft(to_dev(A), precision=prec, out=Ah)
    tube_fft(to_dev(B), precision=prec, out=Bh)
    Ch = fourier_tprod(Ah, Bh, n, s, precision=prec)
    C = torch.empty((4, p, m, s), device=dev)
    tube_fft(Ch, inverse=True, cols=s, out=C)
    assert rel_err(to_np(C), oracle.tprod(A, B)) < TOLS[prec]


@pytest.mark.parametrize("p", [1, 3, 8, 16, 30, 64])
def test_tube_fft_fp64(p):
    X = synth.quat_tensor(5, 9, p, seed=200 + p)
    H = to_np(tube_fft(to_dev(X, torch.float64), precision="fp64"))
    w1 = np.fft.fft(X[0] + 1j * X[1], axis=0)
    w2 = np.fft.fft(X[2] + 1j * X[3], axis=0)
    assert rel_err(H, np.stack([w1.real, w1.imag, w2.real, w2.imag])) < 1e-14


# ------------------------------------------------------------- small configs
def test_c1_fp64():
    A, B = synth.config_inputs(1)
    C = tprod(to_dev(A, torch.float64), to_dev(B, torch.float64), precision="fp64")
    err = rel_err(to_np(C), oracle.tprod(A, B))
    print(f"c1 fp64 rel err {err:.3e}")
    assert err <= FP64_TOL


def test_c1_fp32():
    A, B = synth.config_inputs(1)
    C = tprod(to_dev(A), to_dev(B))
    err = rel_err(to_np(C), oracle.tprod(A, B))
    print(f"c1 fp32 rel err {err:.3e}")
    assert err <= FP32_TOL


# Several GEMM tiles in m and s with ragged tails, several k-chunks with a
# ragged tail, and every kind of p (odd, even, prime factors 2/3/5/7).
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [1, 2, 3, 5, 7, 8, 12, 16, 30, 32])
def test_parity_ragged_full(p, prec):
    m, n, s = 300, 50, 150
    A = synth.quat_tensor(m, n, p, seed=300 + p)
    B = synth.quat_tensor(n, s, p, seed=400 + p)
    C = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
    err = rel_err(C, oracle.tprod_faces(A, B))
    print(f"{prec} p={p} rel err {err:.3e}")
    assert err <= TOLS[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("p", [45, 64, 100, 128])
def test_parity_ragged_faces(p, prec):
    m, n, s = 260, 36, 140
    A = synth.quat_tensor(m, n, p, seed=500 + p)
    B = synth.quat_tensor(n, s, p, seed=600 + p)
    C = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
    faces = [0, 1, p // 2, p - 1]
    err = rel_err(C[:, faces], oracle.tprod_faces(A, B, faces))
    print(f"{prec} p={p} rel err on faces {faces}: {err:.3e}")
    assert err <= TOLS[prec]


@pytest.mark.parametrize("m,n,s,p", [(1, 1, 1, 1), (1, 1, 1, 7), (1, 3, 1, 4), (5, 1, 3, 6),
                                     (2, 2, 2, 2), (129, 17, 65, 3), (128, 16, 64, 4)])
def test_edge_shapes(m, n, s, p):
    A = synth.quat_tensor(m, n, p, seed=700 + m + n + s + p)
    B = synth.quat_tensor(n, s, p, seed=800 + m + n + s + p)
    ref = oracle.tprod(A, B)
    C32 = to_np(tprod(to_dev(A), to_dev(B)))
    assert rel_err(C32, ref) <= FP32_TOL
    for prec in ("split_bf16", "split_fp16"):
        Cs = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
        assert rel_err(Cs, ref) <= SPLIT_GUARD
    C64 = to_np(tprod(to_dev(A, torch.float64), to_dev(B, torch.float64), precision="fp64"))
    assert rel_err(C64, ref) <= FP64_TOL


def test_p1_is_quaternion_matrix_product():
    A = synth.quat_tensor(70, 30, 1, seed=901)
    B = synth.quat_tensor(30, 90, 1, seed=902)
    C = to_np(tprod(to_dev(A), to_dev(B)))
    from oracle.quaternion import qmatmul
    assert rel_err(C[:, 0], qmatmul(A[:, 0], B[:, 0])) <= FP32_TOL


def test_identity_tensor_gpu():
    p, n = 12, 40
    A = synth.quat_tensor(33, n, p, seed=903)
    C = to_np(tprod(to_dev(A), to_dev(oracle.identity(n, p))))
    assert rel_err(C, A) <= FP32_TOL


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic(prec):
    A = synth.quat_tensor(200, 64, 16, seed=904)
    B = synth.quat_tensor(64, 100, 16, seed=905)
    Ad, Bd = to_dev(A), to_dev(B)
    C1 = tprod(Ad, Bd, precision=prec).cpu()
    C2 = tprod(Ad, Bd, precision=prec).cpu()
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("prec", PRECS)
def test_nan_propagates(prec):
    A = synth.quat_tensor(16, 8, 4, seed=906)
    B = synth.quat_tensor(8, 16, 4, seed=907)
    A[1, 2, 3, 4] = np.nan
    C = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
    assert np.isnan(C[:, :, 3, :]).all()          # row 3 of every face is poisoned
    assert np.isfinite(np.delete(C, 3, axis=2)).all()


def test_fp16_scaling_handles_wide_range():
    """Faces spanning 1e-3..1e3 and a tensor of magnitude 1e6: the per-frequency
    power-of-two scales keep fp16 hi/lo in range."""
    m, n, s, p = 96, 40, 70, 12
    w = synth.face_scales(p)[None, :, None, None]
    A = synth.quat_tensor(m, n, p, seed=950) * w * 1e3
    B = synth.quat_tensor(n, s, p, seed=951) * w * 1e3
    C = to_np(tprod(to_dev(A), to_dev(B), precision="split_fp16"))
    err = rel_err(C, oracle.tprod_faces(A, B))
    print(f"fp16 wide range rel err {err:.3e}")
    assert err <= SPLIT_GUARD


@pytest.mark.parametrize("sa,sb", [(1e-17, 1e-17), (1e-20, 1e15), (1e-35, 1e30), (1e15, 1e-20)])
def test_fp16_scaling_tiny_and_mismatched(sa, sb):
    """Operands far from 1 on one or both sides: each frequency's scale is a
    normal power of two (capped at 2^126) and the product is unscaled one
    factor at a time, so tiny operands neither overflow the scale nor the
    unscaling factor."""
    m, n, s, p = 70, 40, 90, 12
    A = synth.quat_tensor(m, n, p, seed=960) * sa
    B = synth.quat_tensor(n, s, p, seed=961) * sb
    ref = oracle.tprod_faces(A, B)
    C = to_np(tprod(to_dev(A), to_dev(B), precision="split_fp16"))
    err = rel_err(C, ref)
    print(f"fp16 scales {sa:g} x {sb:g}: rel err {err:.3e}")
    assert np.isfinite(C).all()
    assert err <= SPLIT_GUARD


def test_status_errors_raise():
    A = to_dev(synth.quat_tensor(4, 4, 4, seed=1))
    with pytest.raises(ValueError):
        tprod(A, to_dev(synth.quat_tensor(5, 4, 4, seed=2)))


# ----------------------------------------------------------- full-size runs
def test_c2_full_size_sampled():
    A, B = synth.config_inputs(2)
    C = to_np(tprod(to_dev(A), to_dev(B)))
    k, i, j = sample_indices(64, 256, 256, 16, seed=2100, per_face=True)
    err = sampled_rel_err(C, A, B, k, i, j)
    print(f"c2 sampled rel err {err:.3e}")
    assert err <= FP32_TOL
    full = oracle.tprod_faces(A, B, [0, 33])
    assert rel_err(C[:, [0, 33]], full) <= FP32_TOL


def _per_face(C, ref_entries, k, p):
    """Sampled error per output face: (max over faces of ||err_face|| / ||ref||
    over all samples, max over faces of ||err_face|| / ||ref_face||)."""
    d2 = np.sum((C - ref_entries) ** 2, axis=0)
    r2 = np.sum(ref_entries ** 2, axis=0)
    fe = np.array([np.sqrt(d2[k == f].sum()) for f in range(p)])
    fr = np.array([np.sqrt(r2[k == f].sum()) for f in range(p)])
    return float(fe.max() / np.sqrt(r2.sum())), float((fe / fr).max())


@pytest.mark.parametrize("draw", [1, 2])
def test_c3_full_size_sampled(draw):
    """1024^3, p = 32 in every float precision.  Draw 2 scales face k of A and
    B by 10^(-3 + 6k/31): the output faces then differ by up to 1e6 in norm.
    The transform mixes all faces, so the rounding error of the Fourier-domain
    products is spread over every output face at the level of the whole
    tensor; a face 1e-6 of the total carries a relative error up to 1e6 times
    the global one (the FP32 CPU FFT form shows the same, ~8e-3 on the
    smallest face).  Gates: whole-tensor relative error, and no single face
    carrying an error above the whole-tensor gate; the per-face relative
    error is printed.  The FP64 test below gates it per face."""
    A, B = synth.config_inputs(3, draw=draw)
    Ad, Bd = to_dev(A), to_dev(B)
    k, i, j = sample_indices(32, 1024, 1024, 12, seed=3100 + draw, per_face=True)
    ref = oracle.tprod_entries(A, B, k, i, j)
    for prec in PRECS:
        C = to_np(tprod(Ad, Bd, precision=prec))[:, k, i, j]
        err = float(np.sqrt(np.sum((C - ref) ** 2)) / np.sqrt(np.sum(ref ** 2)))
        face_vs_all, face_rel = _per_face(C, ref, k, 32)
        print(f"c3 draw {draw} {prec} sampled rel err {err:.3e}; worst face: {face_vs_all:.3e} of the "
              f"total norm, {face_rel:.3e} of its own norm", flush=True)
        assert err <= TOLS[prec]
        assert err <= (SPLIT_GATE if prec.startswith("split") else FP32_TOL)
        assert face_vs_all <= TOLS[prec]


def test_face_scaled_draw_fp64_per_face():
    """The face-scaled draw at 64^3 (p = 32) in FP64, every output face held
    to a relative error of 1e-9 of its own norm (smallest face ~3e-6 of the
    total; FP64 rounding then allows ~1e-11), so a mishandled small face
    cannot hide under the whole-tensor norm.  FP32 on the same inputs: no
    face carries more than the whole-tensor gate."""
    A, B = synth.config_inputs(3, draw=2, scale=16)
    p = A.shape[1]
    ref = oracle.tprod_faces(A, B)
    C64 = to_np(tprod(to_dev(A, torch.float64), to_dev(B, torch.float64), precision="fp64"))
    face_rel = [oracle.rel_frob(C64[:, f], ref[:, f]) for f in range(p)]
    print(f"fp64 face-scaled: global {oracle.rel_frob(C64, ref):.3e}, worst face {max(face_rel):.3e}")
    assert oracle.rel_frob(C64, ref) <= FP64_TOL
    assert max(face_rel) <= 1e-9
    tot = np.sqrt(np.sum(ref ** 2))
    for prec in PRECS:
        C = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
        worst = max(np.sqrt(np.sum((C[:, f] - ref[:, f]) ** 2)) for f in range(p)) / tot
        print(f"{prec} face-scaled 64^3: worst face error {worst:.3e} of the total norm")
        assert oracle.rel_frob(C, ref) <= TOLS[prec] and worst <= TOLS[prec]
