"""Seeded sweep of random shapes and tube lengths through qt_tprod, against
the FP64 oracle: the definition for small p, and for long tubes the
oracle's FFT form of Algorithm 5.1 (pinned against the definition in the
CPU tests).  Lengths cover register-resident 7-smooth p, primes and other
Bluestein lengths up to 4096; shapes are ragged in every dimension."""
import numpy as np
import pytest

import oracle
import synth
from paper_2212_14318_amd import tprod

from gpu_util import rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "split_bf16": 5e-5, "split_fp16": 5e-5}
SMALL_P = [1, 2, 3, 5, 6, 7, 9, 11, 13, 14, 17, 25, 27, 31, 36, 49, 63, 81, 97, 101, 120, 127, 128]
LARGE_P = [200, 257, 500, 1000, 1024, 2048, 4095, 4096]


def _cases():
    rng = np.random.Generator(np.random.PCG64(2718))
    cases = []
    for k in range(24):
        p = int(rng.choice(SMALL_P))
        m, n, s = (int(x) for x in rng.integers(1, 160, 3))
        prec = ["fp32", "split_bf16", "split_fp16"][k % 3]
        cases.append((m, n, s, p, prec, 7000 + k))
    for k, p in enumerate(LARGE_P):
        m, n, s = (int(x) for x in rng.integers(1, 24, 3))
        prec = ["fp32", "split_bf16"][k % 2]
        cases.append((m, n, s, p, prec, 7100 + k))
    return cases


@pytest.mark.parametrize("m,n,s,p,prec,seed", _cases())
def test_random_shape(m, n, s, p, prec, seed):
    A = synth.quat_tensor(m, n, p, seed=seed)
    B = synth.quat_tensor(n, s, p, seed=seed + 50000)
    C = to_np(tprod(to_dev(A), to_dev(B), precision=prec))
    ref = oracle.tprod(A, B) if p <= 128 else oracle.tprod_fft(A, B)
    assert rel_err(C, ref) < TOLS[prec]
