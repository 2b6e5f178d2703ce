"""qt_tprod_noalloc: the allocation-free qt_tprod (its workspace is a fixed
device array inside the library).  Checked through the C-ABI against
qt_tprod on the same inputs (same kernels and plan tables, so bit-identical)
and against the FP64 oracle, on two calls in a row with the second smaller,
so the second call runs on an array that still holds the first call's data."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import ops

from gpu_util import device, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 5e-5, "split_fp16": 5e-5, "fp64": 1e-13}


def _stream():
    return torch.cuda.current_stream(device()).cuda_stream


def _noalloc(A, B, prec):
    _, p, m, n = A.shape
    s = B.shape[3]
    C = torch.full((4, p, m, s), float("nan"), device=A.device, dtype=A.dtype)
    print(f"qt_tprod_noalloc {prec} m={m} n={n} s={s} p={p}", flush=True)
    st = nat.qt_tprod_noalloc(m, n, s, p, A.data_ptr(), B.data_ptr(), C.data_ptr(), nat.PRECISIONS[prec],
                              _stream())
    assert st == nat.QT_OK, nat.qt_status_string(st)
    return C


# p = 23 and 97 take Bluestein transforms, 45 a register-resident one; the
# first call of a p that no earlier call has planned generates the tables in
# the scratch array, later ones use the cached plan.
@pytest.mark.parametrize("prec,shapes", [
    ("fp32", [(70, 40, 50, 23), (30, 20, 25, 23)]),
    ("split_bf16", [(150, 70, 90, 45), (33, 17, 65, 12)]),
    ("split_fp16", [(130, 66, 129, 16), (40, 24, 36, 97)]),
    ("fp64", [(24, 16, 20, 9), (8, 8, 8, 8)]),
])
def test_noalloc_matches_tprod(prec, shapes):
    dt = torch.float64 if prec == "fp64" else torch.float32
    for k, (m, n, s, p) in enumerate(shapes):
        A64 = synth.quat_tensor(m, n, p, seed=4700 + 2 * k)
        B64 = synth.quat_tensor(n, s, p, seed=4701 + 2 * k)
        A, B = to_dev(A64, dt), to_dev(B64, dt)
        C0 = _noalloc(A, B, prec)
        torch.cuda.synchronize()
        C1 = ops.tprod(A, B, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(C0, C1), f"call {k}: noalloc and qt_tprod differ"
        err = rel_err(to_np(C0), oracle.tprod(A64, B64))
        assert err < TOL[prec], f"call {k}: rel. error {err:.3e}"


def test_noalloc_rejects_too_large_before_launch():
    dev = device()
    # 16 p (mn + ns + ms) bytes of workspace: 512 x 512 x 512, p = 32 needs 402 MB
    m = n = s = 512
    p = 32
    assert nat.qt_workspace_size(m, n, s, p, nat.QT_FP32) > nat.QT_NOALLOC_SCRATCH_BYTES
    A = torch.zeros((4, p, m, n), device=dev)
    B = torch.zeros((4, p, n, s), device=dev)
    C = torch.full((4, p, m, s), 7.0, device=dev)
    st = nat.qt_tprod_noalloc(m, n, s, p, A.data_ptr(), B.data_ptr(), C.data_ptr(), nat.QT_FP32, _stream())
    assert st == nat.QT_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())       # nothing ran
