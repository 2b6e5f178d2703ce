"""Quaternion t-SVD, A = U * S * V^H (oracle, FP64; test infrastructure only).

The paper names T-product based factorisations of quaternion tensors as the
next use of its block diagonalisation (Section 6) without giving one, so what
is fixed here is the definition and what follows from Theorem 5.1:

* A (m x n x p) = U * S * V^H with U (m x m x p) and V (n x n x p) unitary
  tensors (U^H * U = U * U^H = identity) and S (m x n x p) f-diagonal (every
  face is a diagonal matrix).  Then bcirc(A) = bcirc(U) bcirc(S) bcirc(V)^*
  with bcirc(U), bcirc(V) unitary, so the singular values of the quaternion
  matrix bcirc(A) are those of bcirc(S).

* The frequency-pair matrices.  With X^1, X^2 the tube DFTs of the complex
  parts of X = X1 + X2 j (plain DFT, exp(-2 pi i f k / p)), put

      chi_f(X) = [[ X^1[f],          X^2[f]         ],
                  [ -conj X^2[-f],   conj X^1[-f]   ]]      (2 rows x 2 cols blocks).

  The coupled facewise products of Theorem 5.1 / Remark 5.1 say exactly that
  chi_f(A * B) = chi_f(A) chi_f(B) for every f, and chi_f(X^H) = chi_f(X)^*.
  chi_-f(X) = J conj(chi_f(X)) J^T with J = [[0, I], [-I, 0]], so each pair
  {f, -f} carries one independent complex matrix, and for the self-paired
  frequencies (f = 0, and p/2 for even p) chi_f(X) is the complex adjoint of
  the quaternion matrix X^1[f] + X^2[f] j.

* The factorisation per pair.  For a pair f != -f take any SVD
  chi_f(A) = P diag(s) Q^* (s sorted descending) and place singular value
  s_2i into diagonal entry i of S^1[f] and s_2i+1 into entry i of S^1[-f]
  (S^2 = 0); the singular vectors go to the matching columns (i and m + i of
  chi_f(U), i and n + i of chi_f(V)).  For a self-paired f the singular
  values of chi_f(A) come in equal pairs and the factors must again be complex
  adjoints of quaternion matrices; the left vector u = (x; y) of a singular
  value then comes with its partner (-conj y; conj x), which is a left vector
  of the same singular value.  This interleaved placement makes the first r
  diagonal tubes of S hold the 2r largest singular values of every chi_f, so
  that truncating to them is the best approximation in the Frobenius norm
  among tensors whose chi_f all have rank <= 2r (Eckart-Young per pair, with
  ||X||_F^2 = 1 / (2p) sum_f ||chi_f(X)||_F^2).

U, S, V are not unique (phases, and any basis of a repeated singular value's
space or of the null spaces); S is (up to rounding).
"""
from __future__ import annotations

import numpy as np

from .tproduct import bcirc


def _complex_parts(X):
    return X[0] + 1j * X[1], X[2] + 1j * X[3]


def complex_adjoint(Q: np.ndarray) -> np.ndarray:
    """Complex adjoint [[Q1, Q2], [-conj Q2, conj Q1]] of a quaternion matrix
    Q = Q1 + Q2 j given as (4, r, c): a (2r, 2c) complex matrix."""
    Q1, Q2 = _complex_parts(np.asarray(Q, dtype=np.float64))
    return np.block([[Q1, Q2], [-np.conj(Q2), np.conj(Q1)]])


def bcirc_singular_values(A: np.ndarray) -> np.ndarray:
    """Singular values of the quaternion matrix bcirc(A), descending
    (p * min(m, n) values).  Each appears twice among those of the complex
    adjoint of bcirc(A); one of each pair is returned."""
    sv = np.linalg.svd(complex_adjoint(bcirc(A)), compute_uv=False)
    return np.sort(sv)[::-1][0::2]


def chi(X: np.ndarray) -> np.ndarray:
    """chi_f(X) for every f: complex array (p, 2 rows, 2 cols)."""
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[1]
    X1, X2 = _complex_parts(X)
    h1, h2 = np.fft.fft(X1, axis=0), np.fft.fft(X2, axis=0)
    neg = (-np.arange(p)) % p
    top = np.concatenate([h1, h2], axis=2)
    bot = np.concatenate([-np.conj(h2[neg]), np.conj(h1[neg])], axis=2)
    return np.concatenate([top, bot], axis=1)


def from_chi(M: np.ndarray, rows: int, cols: int) -> np.ndarray:
    """Quaternion tensor (4, p, rows, cols) whose chi_f is M[f] (the blocks
    X^1[f], X^2[f] are read from the top block row of each chi_f)."""
    h1 = M[:, :rows, :cols]
    h2 = M[:, :rows, cols:]
    X1, X2 = np.fft.ifft(h1, axis=0), np.fft.ifft(h2, axis=0)
    return np.stack([X1.real, X1.imag, X2.real, X2.imag])


def _partner(u: np.ndarray) -> np.ndarray:
    """(x; y) -> (-conj y; conj x): the second column that a quaternion
    column contributes to a complex adjoint."""
    r = u.shape[0] // 2
    return np.concatenate([-np.conj(u[r:]), np.conj(u[:r])])


def _J(d: int) -> np.ndarray:
    """J = [[0, I], [-I, 0]] of size 2d: chi_-f(X) = J conj(chi_f(X)) J^T."""
    return np.block([[np.zeros((d, d)), np.eye(d)], [-np.eye(d), np.zeros((d, d))]])


def _structured_basis(cands, r, start):
    """Extend the partner-closed orthonormal set `start` (list of 2r-vectors)
    by candidates, each taken with its partner, until it has 2r vectors.
    Returns the accepted (first-half) vectors in order."""
    basis = list(start)
    taken = []
    for v in cands:
        if len(basis) >= 2 * r:
            break
        w = v.astype(np.complex128)
        for _ in range(2):                      # Gram-Schmidt, twice
            for b in basis:
                w = w - b * np.vdot(b, w)
        nrm = np.linalg.norm(w)
        if nrm < 1e-6:
            continue
        w = w / nrm
        taken.append(w)
        basis += [w, _partner(w)]
    return taken


def tsvd(A: np.ndarray):
    """t-SVD of A (4, p, m, n): returns U (4, p, m, m), S (4, p, m, n),
    V (4, p, n, n) with A = U * S * V^H, and sigma (p, min(m, n)), the
    diagonal of S^1[f] (the Fourier-domain singular values)."""
    A = np.asarray(A, dtype=np.float64)
    _, p, m, n = A.shape
    k = min(m, n)
    Mf = chi(A)
    CU = np.zeros((p, 2 * m, 2 * m), dtype=np.complex128)
    CV = np.zeros((p, 2 * n, 2 * n), dtype=np.complex128)
    sigma = np.zeros((p, k))
    for f in range(p // 2 + 1):
        g = (-f) % p
        P, s, Qh = np.linalg.svd(Mf[f], full_matrices=True)
        Q = Qh.conj().T
        if f != g:
            # interleave: s_2i -> slot i (frequency f), s_2i+1 -> slot m + i (n + i)
            uslot = [i // 2 + (m if i % 2 else 0) for i in range(2 * k)]
            vslot = [i // 2 + (n if i % 2 else 0) for i in range(2 * k)]
            Uf = np.zeros((2 * m, 2 * m), dtype=np.complex128)
            Vf = np.zeros((2 * n, 2 * n), dtype=np.complex128)
            for i in range(2 * k):
                Uf[:, uslot[i]] = P[:, i]
                Vf[:, vslot[i]] = Q[:, i]
            ufree = [c for c in range(2 * m) if c not in uslot]
            vfree = [c for c in range(2 * n) if c not in vslot]
            for c, col in zip(ufree, range(2 * k, 2 * m)):
                Uf[:, c] = P[:, col]
            for c, col in zip(vfree, range(2 * k, 2 * n)):
                Vf[:, c] = Q[:, col]
            sigma[f] = s[0::2][:k]
            sigma[g] = s[1::2][:k]
            CU[f], CV[f] = Uf, Vf
            CU[g] = _J(m) @ np.conj(Uf) @ _J(m).T
            CV[g] = _J(n) @ np.conj(Vf) @ _J(n).T
        else:
            # quaternion singular vectors: one right vector per equal pair (its
            # partner is the other), left vectors u = chi_f(A) v / s, and the
            # left null space completed with partners as well
            vs = _structured_basis([Q[:, i] for i in range(2 * n)] + list(np.eye(2 * n).T), n, [])
            tiny = 1e-12 * max(float(s[0]), 1e-300) if s.size else 0.0
            us = [None] * m
            for i in range(k):
                w = Mf[f] @ vs[i]
                sigma[f, i] = np.linalg.norm(w)
                if sigma[f, i] > tiny:
                    us[i] = w / sigma[f, i]
            start = []
            for u in us:
                if u is not None:
                    start += [u, _partner(u)]
            extra = iter(_structured_basis([P[:, i] for i in range(2 * m)] + list(np.eye(2 * m).T), m, start))
            us = [u if u is not None else next(extra) for u in us]
            Uf = np.zeros((2 * m, 2 * m), dtype=np.complex128)
            Vf = np.zeros((2 * n, 2 * n), dtype=np.complex128)
            for i in range(m):
                Uf[:, i], Uf[:, m + i] = us[i], _partner(us[i])
            for i in range(n):
                Vf[:, i], Vf[:, n + i] = vs[i], _partner(vs[i])
            CU[f], CV[f] = Uf, Vf
    S = np.zeros((4, p, m, n))
    d = np.arange(k)
    Sd = np.fft.ifft(sigma.astype(np.complex128), axis=0)       # (p, k): tubes of S1's diagonal
    S[0][:, d, d] = Sd.real
    S[1][:, d, d] = Sd.imag
    return from_chi(CU, m, m), S, from_chi(CV, n, n), sigma
