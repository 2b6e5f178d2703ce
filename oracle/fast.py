"""The fast T-product on the CPU (oracle companion, FP64 by default).

Test infrastructure only: the CPU FFT-based version that the benchmark times
beside the definitional oracle, and a second route to A * B that the tests pin
against the definition.  It shares nothing with the GPU path.

What it evaluates (Theorem 4.4 for the transform, Theorem 5.1 and Remark 5.1
for the coupled facewise products, Remark 4.3 for the inverse), written in
the plain-DFT convention.  A quaternion tensor X = X1 + X2 j has the complex
parts X1 = a + b i and X2 = c + d i (Section 2.2).  With F the unnormalised
DFT along the faces (numpy's fft, exp(-2 pi i f k / p)) and F^-1 its inverse
with the factor 1/p:

    X^1 = F X1,  X^2 = F X2                    (every tube, both tensors)
    C^1[f] = A^1[f] B^1[f] - A^2[f] conj(B^2[-f])
    C^2[f] = A^1[f] B^2[f] + A^2[f] conj(B^1[-f])    (-f taken mod p)
    C1 = F^-1 C^1,  C2 = F^-1 C^2.

The coupling of f with -f is what j c = conj(c) j does to a product of two
Cayley-Dickson forms: (X1 + X2 j)(Y1 + Y2 j) = (X1 Y1 - X2 conj Y2) +
(X1 Y2 + X2 conj Y1) j, and the DFT of a conjugated tube is the conjugate of
the spectrum read at -f.  The paper writes the same transform on conj X and
pairs face i with face p + 2 - i; the two conventions give the same C (the
tests check both against the definition).
"""
from __future__ import annotations

import numpy as np


def tprod_fft(A: np.ndarray, B: np.ndarray, dtype=np.complex128) -> np.ndarray:
    """C = A * B through the Fourier domain; A (4, p, m, n), B (4, p, n, s).

    dtype: complex type of the Fourier-domain work (complex128, the oracle
    precision; complex64 gives the single-precision CPU baseline)."""
    if A.ndim != 4 or B.ndim != 4 or A.shape[0] != 4 or B.shape[0] != 4:
        raise ValueError("quaternion tensors must have shape (4, p, rows, cols)")
    if A.shape[1] != B.shape[1] or A.shape[3] != B.shape[2]:
        raise ValueError("A must be m x n x p and B n x s x p")
    p = A.shape[1]
    neg = (-np.arange(p)) % p                          # index of -f for every f

    def spectra(X):
        X1 = (X[0] + 1j * X[1]).astype(dtype)
        X2 = (X[2] + 1j * X[3]).astype(dtype)
        return np.fft.fft(X1, axis=0).astype(dtype), np.fft.fft(X2, axis=0).astype(dtype)

    a1, a2 = spectra(A)
    b1, b2 = spectra(B)
    # all frequencies at once: (p, m, n) @ (p, n, s) is one matrix product per face
    c1 = a1 @ b1 - a2 @ np.conj(b2[neg])
    c2 = a1 @ b2 + a2 @ np.conj(b1[neg])
    del a1, a2, b1, b2
    C1 = np.fft.ifft(c1, axis=0)
    C2 = np.fft.ifft(c2, axis=0)
    return np.stack([C1.real, C1.imag, C2.real, C2.imag])
