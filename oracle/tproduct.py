"""Definitional T-product of third-order quaternion tensors (oracle, FP64).

Test infrastructure only.  Tensors are float64 arrays of shape (4, p, rows, cols)
(component, face, row, column); face r of the paper (1-based, A^(r)) is
X[:, r - 1] here.

Definition (Section 2.4, operators bcirc / unfold / fold and the Definition of
the T-product): for A of size m x n x p and B of size n x s x p,

    bcirc(A)  = the mp x np block matrix whose first block column is
                A^(1), A^(2), ..., A^(p) and whose every other block column is
                the previous one shifted down by one block (cyclically);
    unfold(B) = the np x s block column (B^(1); B^(2); ...; B^(p));
    A * B     = fold( bcirc(A) . unfold(B) ),   of size m x s x p,

where "." is the quaternion matrix product.  In 0-based face indices the block
in block-row k, block-column r of bcirc(A) is A[(k - r) mod p].

Companions that the paper does not define but the method's users need:

* tensor conjugate transpose X^H (the Kilmer-Martin transpose carried over to
  quaternions): face 0 of X^H is the conjugate transpose of face 0 of X, face k
  (k >= 1) of X^H is the conjugate transpose of face p - k of X.  Equivalently
  bcirc(X^H) is the conjugate transpose of bcirc(X).
* identity tensor: face 0 is the identity matrix, all other faces are zero.
* loss L(A, B) = 1/2 ||A * B - T||_F^2 and its adjoints
  dL/dA = G * B^H, dL/dB = A^H * G with G = A * B - T.
"""
from __future__ import annotations

import numpy as np

from .quaternion import qconjT, qmatmul, qmul, qnorm2


def _check(A: np.ndarray, B: np.ndarray):
    if A.ndim != 4 or B.ndim != 4 or A.shape[0] != 4 or B.shape[0] != 4:
        raise ValueError("quaternion tensors must have shape (4, p, rows, cols)")
    if A.shape[1] != B.shape[1]:
        raise ValueError("A and B must have the same number of faces p")
    if A.shape[3] != B.shape[2]:
        raise ValueError("inner dimensions differ: A is m x n x p, B must be n x s x p")


def bcirc(A: np.ndarray) -> np.ndarray:
    """Block circulant matrix of A: shape (4, m p, n p).

    Block (k, r) (0-based block row k, block column r) is face (k - r) mod p.
    """
    A = np.asarray(A, dtype=np.float64)
    _, p, m, n = A.shape
    M = np.empty((4, m * p, n * p), dtype=np.float64)
    for k in range(p):
        for r in range(p):
            M[:, k * m:(k + 1) * m, r * n:(r + 1) * n] = A[:, (k - r) % p]
    return M


def unfold(B: np.ndarray) -> np.ndarray:
    """Stack the faces of B vertically: shape (4, n p, s)."""
    B = np.asarray(B, dtype=np.float64)
    _, p, n, s = B.shape
    return B.reshape(4, p * n, s)


def fold(M: np.ndarray, p: int) -> np.ndarray:
    """Inverse of unfold: (4, m p, s) -> (4, p, m, s)."""
    _, mp, s = M.shape
    if mp % p:
        raise ValueError("row count is not a multiple of p")
    return M.reshape(4, p, mp // p, s)


def tprod(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A * B = fold(bcirc(A) . unfold(B)), materialising bcirc(A).

    Memory is 32 m n p^2 bytes for bcirc(A); use tprod_faces for larger inputs.
    """
    _check(A, B)
    p = A.shape[1]
    return fold(qmatmul(bcirc(A), unfold(B)), p)


def tprod_faces(A: np.ndarray, B: np.ndarray, faces=None) -> np.ndarray:
    """Selected output faces of A * B, one block row of bcirc(A) at a time.

    Face k of fold(bcirc(A) . unfold(B)) is block row k of bcirc(A) times
    unfold(B), i.e. sum over r of A[(k - r) mod p] . B[r].  This is the same
    matrix product as tprod, evaluated block row by block row so that bcirc(A)
    is never stored.  Returns shape (4, len(faces), m, s) (all faces if None).
    """
    _check(A, B)
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    _, p, m, n = A.shape
    s = B.shape[3]
    faces = list(range(p)) if faces is None else [int(k) for k in faces]
    out = np.zeros((4, len(faces), m, s), dtype=np.float64)
    for idx, k in enumerate(faces):
        acc = np.zeros((4, m, s), dtype=np.float64)
        for r in range(p):
            acc += qmatmul(A[:, (k - r) % p], B[:, r])
        out[:, idx] = acc
    return out


def tprod_rows(A: np.ndarray, B: np.ndarray, rows) -> np.ndarray:
    """Selected rows i of every face of A * B: shape (4, p, len(rows), s).

    Row i of face k is sum over r of (row i of A[(k - r) mod p]) . B[r]; this
    restricts the block-row product of tprod_faces to a few matrix rows.
    """
    _check(A, B)
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    p = A.shape[1]
    rows = np.asarray(rows, dtype=np.int64)
    Ar = A[:, :, rows, :]
    out = np.zeros((4, p, len(rows), B.shape[3]), dtype=np.float64)
    for k in range(p):
        for r in range(p):
            out[:, k] += qmatmul(Ar[:, (k - r) % p], B[:, r])
    return out


def tprod_cols(A: np.ndarray, B: np.ndarray, cols) -> np.ndarray:
    """Selected columns j of every face of A * B: shape (4, p, m, len(cols)).

    Column j of face k is sum over r of A[(k - r) mod p] . (column j of B[r]).
    """
    cols = np.asarray(cols, dtype=np.int64)
    return tprod_faces(A, np.asarray(B, dtype=np.float64)[:, :, :, cols])


def tprod_entries(A: np.ndarray, B: np.ndarray, faces, rows, cols) -> np.ndarray:
    """Single entries C[:, k, i, j] of C = A * B for index lists (k, i, j).

    C[k, i, j] = sum over r in [0, p) and l in [0, n) of
                 A[(k - r) mod p, i, l] B[r, l, j]  (Hamilton products),
    which is entry (k m + i, j) of bcirc(A) . unfold(B).  Returns (4, len).
    """
    _check(A, B)
    faces = np.asarray(faces, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    p = A.shape[1]
    out = np.empty((4, faces.size), dtype=np.float64)
    r = np.arange(p)
    for t in range(faces.size):
        k, i, j = faces[t], rows[t], cols[t]
        # A[:, (k - r) mod p, i, :] -> (4, p, n); B[:, r, :, j] -> (p, 4, n) -> (4, p, n)
        a = np.asarray(A[:, (k - r) % p, i, :], dtype=np.float64)
        b = np.moveaxis(np.asarray(B[:, r, :, j], dtype=np.float64), 0, 1)
        out[:, t] = qmul(a, b).sum(axis=(1, 2))
    return out


def tconjT(X: np.ndarray) -> np.ndarray:
    """Tensor conjugate transpose X^H, shape (4, p, cols, rows).

    Face 0 -> (face 0)^*, face k -> (face p - k)^* for k >= 1, with ^* the
    quaternion conjugate transpose.  bcirc(X^H) = bcirc(X)^*.
    """
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[1]
    order = [0] + [p - k for k in range(1, p)]
    return qconjT(X[:, order])


def identity(n: int, p: int) -> np.ndarray:
    """Identity tensor of size n x n x p: face 0 = I_n, other faces zero."""
    I = np.zeros((4, p, n, n), dtype=np.float64)
    I[0, 0] = np.eye(n)
    return I


def loss(A: np.ndarray, B: np.ndarray, T: np.ndarray) -> float:
    """L = 1/2 ||A * B - T||_F^2 over all four real components."""
    return 0.5 * qnorm2(tprod_faces(A, B) - T)


def adjoints(A: np.ndarray, B: np.ndarray, G: np.ndarray):
    """Adjoints of the T-product for an output gradient G.

    For L with dL/dC = G (for the loss above, G = A * B - T):
    dL/dA = G * B^H and dL/dB = A^H * G.  Reason: for the real inner product
    <X, Y> = sum of component products, <G, dA * B> = <G * B^H, dA> and
    <G, A * dB> = <A^H * G, dB>, because bcirc turns * into the matrix
    product, bcirc(X^H) = bcirc(X)^*, and Re tr(PQ) = Re tr(QP) for
    quaternion matrices.
    """
    dA = tprod_faces(G, tconjT(B))
    dB = tprod_faces(tconjT(A), G)
    return dA, dB


def rel_frob(X: np.ndarray, ref: np.ndarray) -> float:
    """Relative Frobenius error ||X - ref||_F / ||ref||_F over all components."""
    X = np.asarray(X, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sqrt(qnorm2(ref))
    num = np.sqrt(qnorm2(X - ref))
    return float(num / den) if den > 0 else float(num)
