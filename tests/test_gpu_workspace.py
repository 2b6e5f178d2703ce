"""Library-allocated workspaces: ws == NULL with ws_bytes == 0 takes the
workspace from the stream-ordered allocator for the call.  The results must
be bit-identical to the same call on a caller-provided workspace (same
kernels, same order), and correct against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import _native as nat
from paper_2212_14318_amd import ops

from gpu_util import device, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream(device()).cuda_stream


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_tprod_null_workspace(prec):
    m, n, s, p = 70, 33, 50, 12
    A, B = synth.quat_tensor(m, n, p, seed=4400), synth.quat_tensor(n, s, p, seed=4401)
    Ad, Bd = to_dev(A), to_dev(B)
    C1 = ops.tprod(Ad, Bd, precision=prec)
    C2 = torch.empty_like(C1)
    st = nat.qt_tprod(m, n, s, p, Ad.data_ptr(), Bd.data_ptr(), C2.data_ptr(), nat.PRECISIONS[prec], None, 0,
                      _stream())
    assert st == nat.QT_OK
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    assert rel_err(to_np(C2), oracle.tprod(A, B)) < 5e-5


def test_backward_null_workspace():
    m, n, s, p = 40, 24, 30, 8
    A, B = synth.quat_tensor(m, n, p, seed=4410), synth.quat_tensor(n, s, p, seed=4411)
    G = synth.quat_tensor(m, s, p, seed=4412)
    Ad, Bd, Gd = to_dev(A), to_dev(B), to_dev(G)
    dA1, dB1 = ops.tprod_backward(Ad, Bd, Gd)
    dA2, dB2 = torch.empty_like(dA1), torch.empty_like(dB1)
    st = nat.qt_tprod_backward(m, n, s, p, Ad.data_ptr(), Bd.data_ptr(), Gd.data_ptr(), dA2.data_ptr(),
                               dB2.data_ptr(), nat.QT_FP32, None, 0, _stream())
    assert st == nat.QT_OK
    torch.cuda.synchronize()
    assert torch.equal(dA1, dA2) and torch.equal(dB1, dB2)
    rA, rB = oracle.adjoints(A, B, G)
    assert rel_err(to_np(dA2), rA) < 1e-5 and rel_err(to_np(dB2), rB) < 1e-5


def test_complex_and_real_null_workspace():
    m, n, s, p = 50, 20, 40, 9
    A = synth.quat_tensor(m, n, p, seed=4420)[:2].copy()
    B = synth.quat_tensor(n, s, p, seed=4421)[:2].copy()
    Ad, Bd = to_dev(A), to_dev(B)
    C1 = ops.tprod_complex(Ad, Bd)
    C2 = torch.empty_like(C1)
    assert nat.qt_tprod_complex(m, n, s, p, Ad.data_ptr(), Bd.data_ptr(), C2.data_ptr(), nat.QT_FP32, None, 0,
                                _stream()) == nat.QT_OK
    R1 = ops.tprod_real(Ad[0], Bd[0])
    R2 = torch.empty_like(R1)
    assert nat.qt_tprod_real(m, n, s, p, Ad[0].data_ptr(), Bd[0].data_ptr(), R2.data_ptr(), nat.QT_FP32, None, 0,
                             _stream()) == nat.QT_OK
    torch.cuda.synchronize()
    assert torch.equal(C1, C2) and torch.equal(R1, R2)


def test_batched_null_workspace():
    sizes = [(40, 17, 33, 8), (16, 64, 20, 12), (70, 30, 9, 5)]
    As, Bs, Cs, refs = [], [], [], []
    for i, (m, n, s, p) in enumerate(sizes):
        A, B = synth.quat_tensor(m, n, p, seed=4430 + i), synth.quat_tensor(n, s, p, seed=4440 + i)
        As.append(to_dev(A)); Bs.append(to_dev(B))
        Cs.append(torch.full((4, p, m, s), float("nan"), device=device()))
        refs.append(oracle.tprod(A, B))
    probs = (nat.qt_problem * len(sizes))()
    for k, ((m, n, s, p), A, B, C) in enumerate(zip(sizes, As, Bs, Cs)):
        probs[k] = nat.qt_problem(m, n, s, p, A.data_ptr(), B.data_ptr(), C.data_ptr())
    assert nat.qt_tprod_batched(len(sizes), probs, nat.QT_FP32, None, 0, _stream()) == nat.QT_OK
    torch.cuda.synchronize()
    for C, ref in zip(Cs, refs):
        assert rel_err(to_np(C), ref) < 1e-5


_FAULT_GPU_CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import torch
from paper_2212_14318_amd import _native as nat
dev = torch.device("cuda:0")
A = torch.randn((4, 8, 20, 12), device=dev)
B = torch.randn((4, 8, 12, 16), device=dev)
C = torch.full((4, 8, 20, 16), 7.0, device=dev)
st = nat.qt_tprod(20, 12, 16, 8, A.data_ptr(), B.data_ptr(), C.data_ptr(), nat.QT_FP32, None, 0,
                  torch.cuda.current_stream(dev).cuda_stream)
torch.cuda.synchronize()
print(st, bool((C == 7.0).all()))
"""


def test_injected_allocation_failure_launches_nothing():
    """With QTPROD_FAULT=alloc the ws == NULL call returns QT_ERR_ALLOC and
    leaves the output untouched (no kernel ran); the same call without it
    succeeds (test_tprod_null_workspace).  A child process, since the variable
    is read once per process."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, QTPROD_FAULT="alloc")
    print("child: qt_tprod with QTPROD_FAULT=alloc", flush=True)
    out = subprocess.run([sys.executable, "-c", _FAULT_GPU_CHILD.format(root=root)], env=env,
                         capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    st, untouched = out.stdout.split()[-2:]
    assert int(st) == nat.QT_ERR_ALLOC and untouched == "True"


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_tprod_workspace_contents_do_not_leak(prec):
    """A caller workspace full of NaN bit patterns gives the same result, bit
    for bit, as a zeroed one: with padded Fourier rows (45 and 33 columns,
    padded to 48 and 36) nothing the products or transforms read comes from
    the workspace's previous contents."""
    m, n, s, p = 37, 45, 33, 10
    A, B = synth.quat_tensor(m, n, p, seed=4450), synth.quat_tensor(n, s, p, seed=4451)
    Ad, Bd = to_dev(A), to_dev(B)
    need = nat.qt_workspace_size(m, n, s, p, nat.PRECISIONS[prec])
    ws_nan = torch.full((need,), 255, dtype=torch.uint8, device=device())
    ws_zero = torch.zeros((need,), dtype=torch.uint8, device=device())
    C1 = ops.tprod(Ad, Bd, precision=prec, ws=ws_nan)
    C2 = ops.tprod(Ad, Bd, precision=prec, ws=ws_zero)
    torch.cuda.synchronize()
    assert torch.isfinite(C1).all()
    assert torch.equal(C1, C2)
    assert rel_err(to_np(C1), oracle.tprod(A, B)) < 5e-5


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
def test_batched_workspace_contents_do_not_leak(prec):
    """The batched path on a workspace full of NaN bit patterns: the same
    results, bit for bit, as on a zeroed one (padded Fourier rows in every
    problem, a p without a batched transform among them)."""
    sizes = [(40, 17, 33, 8), (16, 63, 21, 12), (70, 30, 9, 61)]
    As, Bs, refs = [], [], []
    for i, (m, n, s, p) in enumerate(sizes):
        A, B = synth.quat_tensor(m, n, p, seed=4460 + i), synth.quat_tensor(n, s, p, seed=4470 + i)
        As.append(to_dev(A)); Bs.append(to_dev(B))
        refs.append(oracle.tprod(A, B))
    outs = []
    for fill in (255, 0):
        Cs = [torch.empty((4, p, m, s), device=device()) for (m, n, s, p) in sizes]
        probs = (nat.qt_problem * len(sizes))()
        for k, ((m, n, s, p), A, B, C) in enumerate(zip(sizes, As, Bs, Cs)):
            probs[k] = nat.qt_problem(m, n, s, p, A.data_ptr(), B.data_ptr(), C.data_ptr())
        need = nat.qt_batched_workspace_size(len(sizes), probs, nat.PRECISIONS[prec])
        ws = torch.full((need,), fill, dtype=torch.uint8, device=device())
        assert nat.qt_tprod_batched(len(sizes), probs, nat.PRECISIONS[prec], ws.data_ptr(), need,
                                    _stream()) == nat.QT_OK
        torch.cuda.synchronize()
        outs.append(Cs)
    for C1, C2, ref in zip(outs[0], outs[1], refs):
        assert torch.isfinite(C1).all()
        assert torch.equal(C1, C2)
        assert rel_err(to_np(C1), ref) < 5e-5
