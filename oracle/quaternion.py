"""Quaternion element and matrix algebra in float64 (oracle, test infrastructure).

A quaternion array is a numpy array whose FIRST axis has length 4 and holds
the real components (a, b, c, d) of a + b i + c j + d k.

Hamilton's rules (Section 1; also the quaternion block of Table 1 in
Section 2.2): i^2 = j^2 = k^2 = ijk = -1, ij = -ji = k, jk = -kj = i,
ki = -ik = j.  Multiplying out (a1 + b1 i + c1 j + d1 k)(a2 + b2 i + c2 j + d2 k)
with these rules gives, component by component,

    1 : a1 a2 - b1 b2 - c1 c2 - d1 d2
    i : a1 b2 + b1 a2 + c1 d2 - d1 c2
    j : a1 c2 - b1 d2 + c1 a2 + d1 b2
    k : a1 d2 + b1 c2 - c1 b2 + d1 a2

The conjugate of a + b i + c j + d k is a - b i - c j - d k (Section 2.2,
conjugate of an octonion restricted to quaternions); the conjugate transpose of
a matrix conjugates every entry and transposes (Section 2.1).
"""
from __future__ import annotations

import numpy as np


def qmul(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Element-wise Hamilton product of two broadcastable quaternion arrays."""
    a1, b1, c1, d1 = x[0], x[1], x[2], x[3]
    a2, b2, c2, d2 = y[0], y[1], y[2], y[3]
    return np.stack([
        a1 * a2 - b1 * b2 - c1 * c2 - d1 * d2,
        a1 * b2 + b1 * a2 + c1 * d2 - d1 * c2,
        a1 * c2 - b1 * d2 + c1 * a2 + d1 * b2,
        a1 * d2 + b1 * c2 - c1 * b2 + d1 * a2,
    ])


def qmatmul(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Quaternion matrix product Z = X Y.

    X has shape (4, ..., m, n), Y has shape (4, ..., n, s); the leading batch
    axes broadcast like numpy.matmul.  Entry (i, j) of Z is
    sum_l X[i, l] Y[l, j] with the Hamilton product above, so every real
    component of Z is a sum of four real matrix products.
    """
    a1, b1, c1, d1 = X[0], X[1], X[2], X[3]
    a2, b2, c2, d2 = Y[0], Y[1], Y[2], Y[3]
    mm = np.matmul
    return np.stack([
        mm(a1, a2) - mm(b1, b2) - mm(c1, c2) - mm(d1, d2),
        mm(a1, b2) + mm(b1, a2) + mm(c1, d2) - mm(d1, c2),
        mm(a1, c2) - mm(b1, d2) + mm(c1, a2) + mm(d1, b2),
        mm(a1, d2) + mm(b1, c2) - mm(c1, b2) + mm(d1, a2),
    ])


def qconj(X: np.ndarray) -> np.ndarray:
    """Entry-wise quaternion conjugate: (a, b, c, d) -> (a, -b, -c, -d)."""
    return np.stack([X[0], -X[1], -X[2], -X[3]])


def qconjT(X: np.ndarray) -> np.ndarray:
    """Conjugate transpose of a quaternion matrix (last two axes swapped)."""
    return np.swapaxes(qconj(X), -1, -2)


def qnorm2(X: np.ndarray) -> float:
    """Squared Frobenius norm: sum of the squares of all real components.

    This is the sum of |x|^2 over entries, with |x| the modulus of Section 2.2.
    """
    return float(np.sum(np.asarray(X, dtype=np.float64) ** 2))
