"""The paper's fast T-product on the CPU in FP64 (oracle companion).

Test infrastructure only: the CPU FFT-based version that the benchmark times
beside the definitional oracle, and a second route to A * B that the tests
pin against the definition.  It shares nothing with the GPU path.

Algorithm 5.1, in the paper's own convention (Theorem 4.4 for the transform,
Theorem 5.1 with Remark 5.1 for the facewise products, Remark 4.3 for the
inverse).  A quaternion tensor X = X1 + X2 j has complex parts
X1 = a + b i and X2 = c + d i (Section 2.2).

Step 1.  hat X = fft(conj X) along the third mode.  The quaternion conjugate
         of X1 + X2 j is conj(X1) - X2 j, so hat X1 = fft(conj X1) and
         hat X2 = -fft(X2).
Step 2.  For every face i (1-based; face p + 1 means face 1), with
         r = p + 2 - i:
            hat C1(i) = hat A1(r) hat B1(r) - conj(hat A2(i)) hat B2(r)
            hat C2(i) = conj(hat A1(r)) hat B2(i) + hat A2(i) hat B1(i)
         (equations TC and TC2 of Remark 5.1).
Step 3.  C = ifft(conj hat C), where conj hat C = conj(hat C1) - hat C2 j, so
         C1 = ifft(conj hat C1) and C2 = -ifft(hat C2).

numpy's fft is the unnormalised DFT with exp(-2 pi i f k / p) and its ifft
carries 1/p, which is the fft / ifft pair the algorithm names.
"""
from __future__ import annotations

import numpy as np


def _parts(X: np.ndarray):
    return X[0] + 1j * X[1], X[2] + 1j * X[3]


def tprod_fft(A: np.ndarray, B: np.ndarray, dtype=np.complex128) -> np.ndarray:
    """C = A * B by Algorithm 5.1; A (4, p, m, n), B (4, p, n, s).

    dtype: complex type of the Fourier-domain work (complex128, the oracle
    precision; complex64 gives the single-precision CPU baseline)."""
    if A.ndim != 4 or B.ndim != 4 or A.shape[0] != 4 or B.shape[0] != 4:
        raise ValueError("quaternion tensors must have shape (4, p, rows, cols)")
    if A.shape[1] != B.shape[1] or A.shape[3] != B.shape[2]:
        raise ValueError("A must be m x n x p and B n x s x p")
    p = A.shape[1]
    A1, A2 = (x.astype(dtype) for x in _parts(A))
    B1, B2 = (x.astype(dtype) for x in _parts(B))
    # Step 1
    hA1, hA2 = np.fft.fft(np.conj(A1), axis=0), -np.fft.fft(A2, axis=0)
    hB1, hB2 = np.fft.fft(np.conj(B1), axis=0), -np.fft.fft(B2, axis=0)
    # Step 2 (0-based face f = i - 1; r - 1 = (p + 1 - i) mod p = (-f) mod p)
    m, s = A.shape[2], B.shape[3]
    hC1 = np.empty((p, m, s), dtype)
    hC2 = np.empty((p, m, s), dtype)
    for f in range(p):
        r = (-f) % p
        hC1[f] = hA1[r] @ hB1[r] - np.conj(hA2[f]) @ hB2[r]
        hC2[f] = np.conj(hA1[r]) @ hB2[f] + hA2[f] @ hB1[f]
    # Step 3
    C1 = np.fft.ifft(np.conj(hC1), axis=0)
    C2 = -np.fft.ifft(hC2, axis=0)
    return np.stack([C1.real, C1.imag, C2.real, C2.imag])
