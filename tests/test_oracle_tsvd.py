"""Pins of the oracle's quaternion t-SVD (CPU).

The t-SVD is not unique (U and V carry phases and bases of repeated or null
singular spaces), so the pins check what the factorisation must satisfy,
each through a route that does not use the oracle's own frequency-pair
matrices: the definitional T-product (reconstruction, unitarity), the
singular values of the quaternion matrix bcirc(A) computed from the definition
(through its complex adjoint, and for p = 1 through the real 4 x 4 embedding),
the real (Kilmer-Martin) and complex special cases, band-limited tensors for
the pairing of f with -f, and the Frobenius error of truncations.  Planted
mistakes in the oracle must fail at least one pin."""
import numpy as np
import pytest

import oracle
import synth
from oracle import tsvd as ts

SHAPES = [(5, 3, 4), (3, 5, 5), (4, 4, 1), (6, 2, 2), (3, 3, 7), (1, 1, 3), (2, 7, 6), (4, 3, 8)]


def _qr(X):
    """Real 4x4-block embedding of a quaternion matrix (4, r, c): each entry
    a + b i + c j + d k becomes the matrix of left multiplication by it on
    (1, i, j, k) coordinates (Hamilton's rules)."""
    a, b, c, d = X
    return np.block([[a, -b, -c, -d], [b, a, -d, c], [c, d, a, -b], [d, -c, b, a]])


def _checks(A, tol=1e-11):
    """Every pin on one tensor; returns a dict name -> bool."""
    _, p, m, n = A.shape
    k = min(m, n)
    U, S, V, sig = ts.tsvd(A)
    nrm = np.sqrt(oracle.qnorm2(A))
    out = {}
    USVh = oracle.tprod(oracle.tprod(U, S), oracle.tconjT(V))
    out["reconstruction"] = np.sqrt(oracle.qnorm2(USVh - A)) <= tol * nrm
    out["unitary"] = all(
        oracle.rel_frob(oracle.tprod(X, Y), oracle.identity(X.shape[2], p)) <= tol
        for X, Y in ((oracle.tconjT(U), U), (U, oracle.tconjT(U)), (oracle.tconjT(V), V),
                     (V, oracle.tconjT(V))))
    off = S.copy()
    d = np.arange(k)
    off[:2][:, :, d, d] = 0
    out["f_diagonal"] = bool(np.all(off == 0))
    # singular values of bcirc(A) from the definition
    sv = ts.bcirc_singular_values(A)
    got = np.sort(sig.ravel())[::-1]
    out["bcirc_singular_values"] = np.allclose(got, sv, rtol=0, atol=tol * max(sv[0], 1))
    # the diagonal of S's spectrum is sigma
    Shat = np.fft.fft(S[0] + 1j * S[1], axis=0)[:, d, d]
    out["sigma_is_S_spectrum"] = np.allclose(Shat, sig, atol=tol * max(sv[0], 1))
    # pairing of f with -f: a tensor band-limited to {f, -f} has exactly the
    # singular values placed on f and -f
    ok = True
    for f in range(p // 2 + 1):
        g = (-f) % p
        mask = np.zeros(p)
        mask[[f, g]] = 1
        Af = np.real(np.fft.ifft(np.fft.fft(A, axis=1) * mask[None, :, None, None], axis=1))
        want = ts.bcirc_singular_values(Af)[: (2 * k if f != g else k)]
        have = np.sort(np.concatenate([sig[f], sig[g]]) if f != g else sig[f])[::-1]
        ok &= np.allclose(have, want, atol=tol * max(sv[0], 1))
    out["pairs"] = bool(ok)
    # interleaving: sig[f][i] >= sig[-f][i] >= sig[f][i + 1] for 0 < f < p/2
    ok = True
    for f in range(1, (p + 1) // 2):
        a, b = sig[f], sig[(-f) % p]
        ok &= bool(np.all(a >= b - 1e-12)) and bool(np.all(b[:-1] >= a[1:] - 1e-12))
        ok &= bool(np.all(np.diff(a) <= 1e-12))
    out["interleaved"] = bool(ok)
    # truncation: keeping diagonal tubes 0..r-1 of S leaves the error
    # (1 / p) * sum of the squared dropped Fourier singular values, since
    # ||bcirc(X)||_F^2 = p ||X||_F^2 and bcirc(U), bcirc(V) are unitary
    ok = True
    for r in range(k):
        Sr = S.copy()
        Sr[:, :, r:, :] = 0
        Ar = oracle.tprod(oracle.tprod(U, Sr), oracle.tconjT(V))
        err2 = oracle.qnorm2(A - Ar)
        ok &= abs(err2 - np.sum(sig[:, r:] ** 2) / p) <= tol * nrm ** 2
    out["truncation"] = bool(ok)
    return out


@pytest.mark.parametrize("m,n,p", SHAPES)
def test_tsvd_pins(m, n, p):
    A = synth.quat_tensor(m, n, p, seed=7000 + 100 * m + 10 * n + p)
    res = _checks(A)
    assert all(res.values()), res


def test_rank_deficient_and_zero():
    # A = X * Y with inner size 2: chi_f(A) has rank <= 4 < 2 min(m, n)
    X = synth.quat_tensor(6, 2, 5, seed=7101)
    Y = synth.quat_tensor(2, 5, 5, seed=7102)
    A = oracle.tprod(X, Y)
    res = _checks(A, tol=1e-10)
    assert all(res.values()), res
    U, S, V, sig = ts.tsvd(A)
    assert np.all(sig[:, 2:] <= 1e-10 * sig.max())
    Z = np.zeros((4, 4, 3, 2))
    res = _checks(Z)
    assert res["unitary"] and res["reconstruction"] and res["f_diagonal"]


def test_p1_is_quaternion_matrix_svd():
    """p = 1: the singular values of a quaternion matrix, each appearing four
    times among those of its real 4m x 4n embedding."""
    for m, n in ((5, 3), (3, 6), (4, 4)):
        A = synth.quat_tensor(m, n, 1, seed=7200 + m * n)
        sig = ts.tsvd(A)[3][0]
        real_sv = np.linalg.svd(_qr(A[:, 0]), compute_uv=False)
        np.testing.assert_allclose(sig, np.sort(real_sv)[::-1][0::4], atol=1e-12)


def test_real_tensor_is_kilmer_martin_tsvd():
    """A real tensor: chi_f(A) = diag(A^[f], A^[f]), so the Fourier singular
    values are those of each face of numpy's FFT (the real t-SVD)."""
    A = np.zeros((4, 6, 5, 3))
    A[0] = synth.quat_tensor(5, 3, 6, seed=7300)[0]
    sig = ts.tsvd(A)[3]
    want = np.linalg.svd(np.fft.fft(A[0], axis=0), compute_uv=False)
    np.testing.assert_allclose(sig, want, atol=1e-12)


def test_complex_tensor_mixes_f_and_minus_f():
    """A complex tensor (no j part): chi_f(A) = diag(A^[f], conj A^[-f]), so
    the pair {f, -f} shares the singular values of A^[f] and A^[-f]."""
    p = 5
    A = np.zeros((4, p, 4, 3))
    A[:2] = synth.quat_tensor(4, 3, p, seed=7400)[:2]
    sig = ts.tsvd(A)[3]
    h = np.fft.fft(A[0] + 1j * A[1], axis=0)
    for f in range(1, 3):
        g = p - f
        both = np.sort(np.concatenate([np.linalg.svd(h[f], compute_uv=False),
                                       np.linalg.svd(h[g], compute_uv=False)]))[::-1]
        np.testing.assert_allclose(sig[f], both[0::2], atol=1e-12)
        np.testing.assert_allclose(sig[g], both[1::2], atol=1e-12)


def test_chi_is_a_homomorphism():
    """chi_f(A * B) = chi_f(A) chi_f(B) (Theorem 5.1 / Remark 5.1 restated) and
    chi_f(X^H) = chi_f(X)^*, against the definitional T-product."""
    A = synth.quat_tensor(4, 3, 6, seed=7500)
    B = synth.quat_tensor(3, 5, 6, seed=7501)
    np.testing.assert_allclose(ts.chi(oracle.tprod(A, B)), ts.chi(A) @ ts.chi(B), atol=1e-12)
    np.testing.assert_allclose(ts.chi(oracle.tconjT(A)), np.conj(np.swapaxes(ts.chi(A), 1, 2)),
                               atol=1e-12)


# --------------------------------------------------------- planted mistakes
def _mut_chi_uncoupled(X):
    """chi without the -f coupling: the bottom blocks read frequency f."""
    X = np.asarray(X, dtype=np.float64)
    X1, X2 = X[0] + 1j * X[1], X[2] + 1j * X[3]
    h1, h2 = np.fft.fft(X1, axis=0), np.fft.fft(X2, axis=0)
    top = np.concatenate([h1, h2], axis=2)
    bot = np.concatenate([-np.conj(h2), np.conj(h1)], axis=2)
    return np.concatenate([top, bot], axis=1)


def _mut_partner_sign(u):
    r = u.shape[0] // 2
    return np.concatenate([np.conj(u[r:]), np.conj(u[:r])])


def _mut_from_chi_conj(M, rows, cols):
    h1 = np.conj(M[:, :rows, :cols])
    h2 = M[:, :rows, cols:]
    X1, X2 = np.fft.ifft(h1, axis=0), np.fft.ifft(h2, axis=0)
    return np.stack([X1.real, X1.imag, X2.real, X2.imag])


_orig_tsvd = ts.tsvd


def _mut_tsvd_halves(A):
    """Non-interleaved placement: the larger half of each pair's singular
    values all on f, the smaller on -f (re-derived from the correct result)."""
    U, S, V, sig = _orig_tsvd(A)
    p, k = sig.shape
    sig2 = sig.copy()
    for f in range(1, (p + 1) // 2):
        g = p - f
        both = np.sort(np.concatenate([sig[f], sig[g]]))[::-1]
        sig2[f], sig2[g] = both[:k], both[k:]
    S2 = np.zeros_like(S)
    d = np.arange(k)
    Sd = np.fft.ifft(sig2.astype(np.complex128), axis=0)
    S2[0][:, d, d], S2[1][:, d, d] = Sd.real, Sd.imag
    return U, S2, V, sig2


@pytest.mark.parametrize("target,mutant", [
    ("chi", _mut_chi_uncoupled),
    ("_partner", _mut_partner_sign),
    ("from_chi", _mut_from_chi_conj),
    ("tsvd", _mut_tsvd_halves),
])
def test_planted_tsvd_mistakes_are_caught(monkeypatch, target, mutant):
    A = synth.quat_tensor(4, 3, 6, seed=7600)
    assert all(_checks(A).values())
    monkeypatch.setattr(ts, target, mutant)
    assert not all(_checks(A).values())
