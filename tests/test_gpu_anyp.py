"""Any p: lengths without a register-resident tube FFT go through Bluestein's
algorithm.  Checked against numpy's FFT and the FP64 oracle, including the
shapes of the paper's own experiment (Example 5.1, Table 2: m = n = s = 50
with p up to 200 and m = n = s = 100 with p up to 100; the paper reports
relative errors of 4e-17 .. 2.1e-16 for the fast algorithm in FP64)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2212_14318_amd import tprod, tube_fft

from gpu_util import rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


def _want(X):
    w1 = np.fft.fft(X[0] + 1j * X[1], axis=0)
    w2 = np.fft.fft(X[2] + 1j * X[3], axis=0)
    return np.stack([w1.real, w1.imag, w2.real, w2.imag])


@pytest.mark.parametrize("p", [11, 13, 17, 22, 31, 61, 97, 101, 127, 131, 200, 256, 509, 1021, 4096])
def test_bluestein_fp32_matches_numpy(p):
    rows, cols = (3, 21) if p > 1000 else (7, 45)
    X = synth.quat_tensor(rows, cols, p, seed=1200 + p)
    H = to_np(tube_fft(to_dev(X)))
    err = rel_err(H, _want(X))
    back = to_np(tube_fft(to_dev(_want(X)), inverse=True))
    err_b = rel_err(back, X)
    print(f"p={p}: forward {err:.2e}, round trip {err_b:.2e}")
    assert err < 5e-6 and err_b < 5e-6


@pytest.mark.parametrize("p", [11, 65, 97, 128, 200, 1000])
def test_bluestein_fp64_matches_numpy(p):
    X = synth.quat_tensor(5, 19, p, seed=1300 + p)
    H = to_np(tube_fft(to_dev(X, torch.float64), precision="fp64"))
    assert rel_err(H, _want(X)) < 1e-13
    back = to_np(tube_fft(to_dev(_want(X), torch.float64), inverse=True, precision="fp64"))
    assert rel_err(back, X) < 1e-13


@pytest.mark.parametrize("prec", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("p", [11, 13, 37])
def test_tprod_prime_p(prec, p):
    m, n, s = 150, 40, 90
    A = synth.quat_tensor(m, n, p, seed=1400 + p)
    B = synth.quat_tensor(n, s, p, seed=1500 + p)
    C = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
    err = rel_err(C, oracle.tprod_faces(A, B))
    print(f"{prec} p={p}: {err:.3e}")
    assert err <= (1e-5 if prec == "fp32" else 5e-5)


@pytest.mark.parametrize("mns,p", [(50, 10), (50, 50), (50, 100), (50, 200), (100, 10), (100, 50), (100, 100)])
def test_paper_table2_shapes_fp64(mns, p):
    A = synth.quat_tensor(mns, mns, p, seed=1600 + p + mns)
    B = synth.quat_tensor(mns, mns, p, seed=1700 + p + mns)
    C = to_np(tprod(to_dev(A, torch.float64), to_dev(B, torch.float64), precision="fp64"))
    faces = sorted({0, 1, p // 2, p - 1})
    err = rel_err(C[:, faces], oracle.tprod_faces(A, B, faces))
    print(f"({mns},{mns},{mns}) p={p} FP64: {err:.3e}")
    assert err <= 1e-13
