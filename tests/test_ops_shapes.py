"""Host-side checks of the torch wrappers: every wrongly shaped operand is
rejected with ValueError before the C-ABI sees a pointer (the library cannot
know buffer sizes, so a wrong shape would otherwise become an out-of-bounds
device access).  CPU tensors are used: the shape checks come before the
device check, so a correct shape gets as far as "must live on a ROCm device"."""
import pytest
import torch

from paper_2212_14318_amd import ops


def q(p, rows, cols, planes=4, dtype=torch.float32):
    return torch.zeros((planes, p, rows, cols), dtype=dtype)


def raises_shape(fn, *args, **kw):
    with pytest.raises(ValueError) as ei:
        fn(*args, **kw)
    msg = str(ei.value)
    assert "shape" in msg or "cols must be" in msg or "dimension" in msg, msg


def raises_device(fn, *args, **kw):
    with pytest.raises(ValueError, match="ROCm device"):
        fn(*args, **kw)


def test_tprod_shapes():
    A, B = q(5, 3, 4), q(5, 4, 6)
    raises_device(ops.tprod, A, B)
    raises_shape(ops.tprod, A, q(5, 3, 6))                 # B rows != n
    raises_shape(ops.tprod, A, q(4, 4, 6))                 # B faces != p
    raises_shape(ops.tprod, A, B, out=q(5, 3, 7))          # out cols != s
    raises_shape(ops.tprod, A, B, out=q(5, 2, 6))          # out rows != m
    raises_shape(ops.tprod, A, B, out=q(6, 3, 6))          # out faces != p


def test_tube_fft_shapes():
    X = q(5, 3, 8)
    raises_device(ops.tube_fft, X)
    raises_shape(ops.tube_fft, X, out=q(5, 3, 7))          # out narrower than cols
    raises_shape(ops.tube_fft, X, out=q(4, 3, 8))          # p differs
    raises_shape(ops.tube_fft, X, out=q(5, 2, 8))          # rows differ
    raises_shape(ops.tube_fft, X, cols=9)                  # cols beyond the row stride
    raises_shape(ops.tube_fft, X, cols=0)


def test_fourier_tprod_shapes():
    Ah, Bh = q(5, 3, 8), q(5, 6, 8)
    raises_device(ops.fourier_tprod, Ah, Bh, 6, 7)
    raises_shape(ops.fourier_tprod, Ah, Bh, 9, 7)          # n beyond Ah's row stride
    raises_shape(ops.fourier_tprod, Ah, q(5, 5, 8), 6, 7)  # Bh rows != n
    raises_shape(ops.fourier_tprod, Ah, q(4, 6, 8), 6, 7)  # Bh faces != p
    raises_shape(ops.fourier_tprod, Ah, Bh, 6, 9)          # s beyond Bh's row stride
    raises_shape(ops.fourier_tprod, Ah, Bh, 6, 7, out=q(5, 3, 4))   # out narrower than s
    raises_shape(ops.fourier_tprod, Ah, Bh, 6, 7, out=q(5, 2, 8))   # out rows != m


def test_split_words_shapes():
    raises_shape(ops.split_words, q(3, 2, 8), cols=9)


def test_complex_and_real_shapes():
    A, B = q(5, 3, 4, planes=2), q(5, 4, 6, planes=2)
    raises_device(ops.tprod_complex, A, B)
    raises_shape(ops.tprod_complex, A, q(5, 3, 6, planes=2))
    raises_shape(ops.tprod_complex, A, B, out=q(5, 3, 5, planes=2))
    Ar, Br = torch.zeros((5, 3, 4)), torch.zeros((5, 4, 6))
    raises_device(ops.tprod_real, Ar, Br)
    raises_shape(ops.tprod_real, Ar, torch.zeros((5, 3, 6)))
    raises_shape(ops.tprod_real, Ar, Br, out=torch.zeros((5, 3, 5)))


def test_backward_shapes():
    A, B, G = q(5, 3, 4), q(5, 4, 6), q(5, 3, 6)
    raises_device(ops.tprod_backward, A, B, G)
    raises_shape(ops.tprod_backward, A, q(5, 3, 6), G)     # B rows != n
    raises_shape(ops.tprod_backward, A, B, q(5, 3, 5))     # G cols != s
    raises_shape(ops.tprod_backward, A, B, q(4, 3, 6))     # G faces != p


def test_batched_shapes():
    A, B = q(5, 3, 4), q(5, 4, 6)
    raises_device(ops.tprod_batched, [A], [B])
    raises_shape(ops.tprod_batched, [A], [q(5, 3, 6)])
    raises_shape(ops.tprod_batched, [A], [B], outs=[q(5, 3, 5)])
    with pytest.raises(ValueError, match="one output tensor per problem"):
        ops.tprod_batched([A, A], [B, B], outs=[q(5, 3, 6)])
    raises_shape(ops.BatchedPlan, [A], [B], outs=[q(5, 2, 6)])
