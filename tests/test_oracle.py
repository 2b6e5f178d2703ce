"""Pins for the FP64 oracle (CPU only).

Each test checks the oracle against something other than itself: the paper's
multiplication rules and worked example, brute force written from a different
construction of bcirc, textbook reductions (complex adjoint representation and
the FFT-based T-product of complex tensors, Algorithm 2.1), closed forms and
algebraic invariants.  The last test plants plausible mistakes in the oracle
and shows that these pins catch every one of them.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import quaternion as oq
from oracle import tproduct as ot

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_q(rng, *shape):
    return rng.standard_normal((4,) + shape)


# ---------------------------------------------------------------------------
# Independent helpers (not the oracle's code paths)
# ---------------------------------------------------------------------------

# Products of the basis units 1, i, j, k (index 0..3) exactly as the rules of
# Section 1 state them: i^2 = j^2 = k^2 = -1, ij = -ji = k, jk = -kj = i,
# ki = -ik = j.  Entry [a][b] = (sign, index) of e_a e_b.
UNIT = {
    (0, 0): (1, 0), (0, 1): (1, 1), (0, 2): (1, 2), (0, 3): (1, 3),
    (1, 0): (1, 1), (2, 0): (1, 2), (3, 0): (1, 3),
    (1, 1): (-1, 0), (2, 2): (-1, 0), (3, 3): (-1, 0),
    (1, 2): (1, 3), (2, 1): (-1, 3),
    (2, 3): (1, 1), (3, 2): (-1, 1),
    (3, 1): (1, 2), (1, 3): (-1, 2),
}


def brute_qmul(x, y):
    """Scalar quaternion product by distributing over the unit table."""
    out = [0.0, 0.0, 0.0, 0.0]
    for a in range(4):
        for b in range(4):
            sgn, c = UNIT[(a, b)]
            out[c] += sgn * x[a] * y[b]
    return out


def brute_tprod(A, B):
    """fold(bcirc(A) . unfold(B)) with scalar loops.

    bcirc is built as the picture of Section 2.4 draws it: the first block
    row is (A1, Ap, A(p-1), ..., A2) and each following block row is the
    previous one cyclically shifted right by one block.
    """
    _, p, m, n = A.shape
    s = B.shape[3]
    row = [0] + list(range(p - 1, 0, -1))           # face indices of block row 0
    rows = [row]
    for _ in range(1, p):
        prev = rows[-1]
        rows.append([prev[-1]] + prev[:-1])          # cyclic right shift
    C = np.zeros((4, p, m, s))
    for K in range(p):                               # block row
        for R in range(p):                           # block column
            f = rows[K][R]
            for i in range(m):
                for j in range(s):
                    acc = [0.0] * 4
                    for l in range(n):
                        q = brute_qmul(A[:, f, i, l], B[:, R, l, j])
                        for c in range(4):
                            acc[c] += q[c]
                    C[:, K, i, j] += acc
    return C


def chi(X):
    """Complex adjoint representation [[X1, X2], [-conj X2, conj X1]] per face.

    X = X1 + X2 j with X1 = a + b i, X2 = c + d i (Cayley-Dickson form,
    Section 2.2).  chi is a ring homomorphism from quaternion matrices to
    complex matrices (textbook fact), applied to every face.
    """
    X1 = X[0] + 1j * X[1]
    X2 = X[2] + 1j * X[3]
    top = np.concatenate([X1, X2], axis=-1)
    bot = np.concatenate([-np.conj(X2), np.conj(X1)], axis=-1)
    return np.concatenate([top, bot], axis=-2)


def unchi(Z, m, s):
    X1 = Z[..., :m, :s]
    X2 = Z[..., :m, s:]
    return np.stack([X1.real, X1.imag, X2.real, X2.imag])


def complex_tprod_fft(A, B):
    """T-product of complex tensors (faces on axis 0) by Algorithm 2.1."""
    Ah = np.fft.fft(A, axis=0)
    Bh = np.fft.fft(B, axis=0)
    return np.fft.ifft(Ah @ Bh, axis=0)


def cd_planes(X):
    return X[0] + 1j * X[1], X[2] + 1j * X[3]


def from_cd(C1, C2):
    return np.stack([C1.real, C1.imag, C2.real, C2.imag])


# ---------------------------------------------------------------------------
# Element algebra
# ---------------------------------------------------------------------------

def test_hamilton_rules_from_paper():
    """qmul reproduces i^2 = j^2 = k^2 = ijk = -1, ij = k, jk = i, ki = j."""
    e = np.eye(4)
    one, i, j, k = e[0], e[1], e[2], e[3]
    q = lambda x, y: oq.qmul(x[:, None], y[:, None])[:, 0]
    np.testing.assert_array_equal(q(i, i), -one)
    np.testing.assert_array_equal(q(j, j), -one)
    np.testing.assert_array_equal(q(k, k), -one)
    np.testing.assert_array_equal(q(q(i, j), k), -one)
    np.testing.assert_array_equal(q(i, j), k)
    np.testing.assert_array_equal(q(j, i), -k)
    np.testing.assert_array_equal(q(j, k), i)
    np.testing.assert_array_equal(q(k, j), -i)
    np.testing.assert_array_equal(q(k, i), j)
    np.testing.assert_array_equal(q(i, k), -j)


def test_qmul_matches_unit_table(rng):
    x = rng.standard_normal((4, 50))
    y = rng.standard_normal((4, 50))
    got = oq.qmul(x, y)
    for t in range(50):
        np.testing.assert_allclose(got[:, t], brute_qmul(x[:, t], y[:, t]), rtol=0, atol=1e-14)


def test_cd_rule_j_c_equals_conj_c_j(rng):
    """j c = conj(c) j for complex c (Section 1 and Example 3.1)."""
    c = rng.standard_normal((4, 20))
    c[2:] = 0.0                       # complex: a + b i
    jj = np.zeros((4, 20)); jj[2] = 1.0
    np.testing.assert_allclose(oq.qmul(jj, c), oq.qmul(oq.qconj(c), jj), atol=1e-15)


def test_qmatmul_is_chi_homomorphism(rng):
    """chi(X Y) = chi(X) chi(Y): pins qmatmul against complex matmul."""
    X = rand_q(rng, 5, 7)
    Y = rand_q(rng, 7, 3)
    Z = oq.qmatmul(X, Y)
    np.testing.assert_allclose(chi(Z), chi(X) @ chi(Y), atol=1e-12)


def test_norm_is_sum_of_moduli(rng):
    X = rand_q(rng, 3, 4)
    mod2 = sum(oq.qmul(oq.qconj(X[:, i:i + 1, j:j + 1]), X[:, i:i + 1, j:j + 1])[0, 0, 0]
               for i in range(3) for j in range(4))
    assert abs(oq.qnorm2(X) - mod2) < 1e-12


# ---------------------------------------------------------------------------
# Definitional T-product
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,s,p", [(1, 1, 1, 1), (2, 3, 2, 1), (2, 2, 3, 2),
                                     (3, 2, 2, 3), (2, 3, 1, 4), (1, 2, 3, 5)])
def test_brute_force(rng, m, n, s, p):
    A = rand_q(rng, p, m, n)
    B = rand_q(rng, p, n, s)
    ref = brute_tprod(A, B)
    np.testing.assert_allclose(ot.tprod(A, B), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ot.tprod_faces(A, B), ref, rtol=0, atol=1e-12)
    k = rng.integers(0, p, 10); i = rng.integers(0, m, 10); j = rng.integers(0, s, 10)
    np.testing.assert_allclose(ot.tprod_entries(A, B, k, i, j), ref[:, k, i, j], atol=1e-12)
    rows = np.array(sorted(set(rng.integers(0, m, 2).tolist())))
    np.testing.assert_allclose(ot.tprod_rows(A, B, rows), ref[:, :, rows, :], atol=1e-12)
    cols = np.array(sorted(set(rng.integers(0, s, 2).tolist())))
    np.testing.assert_allclose(ot.tprod_cols(A, B, cols), ref[:, :, :, cols], atol=1e-12)


def test_bcirc_picture(rng):
    """First block column is A1..Ap; first block row is A1, Ap, ..., A2."""
    A = rand_q(rng, 4, 2, 3)
    M = ot.bcirc(A)
    for r in range(4):
        np.testing.assert_array_equal(M[:, r * 2:(r + 1) * 2, 0:3], A[:, r])
    expect_row = [0, 3, 2, 1]
    for c in range(4):
        np.testing.assert_array_equal(M[:, 0:2, c * 3:(c + 1) * 3], A[:, expect_row[c]])


def test_p1_is_quaternion_matrix_product(rng):
    A = rand_q(rng, 1, 6, 4)
    B = rand_q(rng, 1, 4, 5)
    C = ot.tprod(A, B)
    Z = chi(C[:, 0])
    np.testing.assert_allclose(Z, chi(A[:, 0]) @ chi(B[:, 0]), atol=1e-12)


def test_single_face_closed_form(rng):
    """A with only face a, B with only face b -> C only at face (a + b) mod p."""
    p, m, n, s = 7, 3, 4, 2
    for a, b in [(0, 0), (2, 3), (5, 4), (6, 6)]:
        A = np.zeros((4, p, m, n)); A[:, a] = rand_q(rng, m, n)
        B = np.zeros((4, p, n, s)); B[:, b] = rand_q(rng, n, s)
        C = ot.tprod_faces(A, B)
        f = (a + b) % p
        for k in range(p):
            if k == f:
                np.testing.assert_allclose(chi(C[:, k]), chi(A[:, a]) @ chi(B[:, b]), atol=1e-12)
            else:
                assert np.all(C[:, k] == 0.0)


def test_identity_tensor(rng):
    p, m, n = 5, 4, 3
    A = rand_q(rng, p, m, n)
    np.testing.assert_allclose(ot.tprod(ot.identity(m, p), A), A, atol=1e-14)
    np.testing.assert_allclose(ot.tprod(A, ot.identity(n, p)), A, atol=1e-14)


def test_associativity(rng):
    p = 6
    A, B, C = rand_q(rng, p, 3, 4), rand_q(rng, p, 4, 2), rand_q(rng, p, 2, 5)
    left = ot.tprod(ot.tprod(A, B), C)
    right = ot.tprod(A, ot.tprod(B, C))
    assert ot.rel_frob(left, right) < 1e-13


def test_not_commutative(rng):
    p = 3
    A, B = rand_q(rng, p, 3, 3), rand_q(rng, p, 3, 3)
    assert ot.rel_frob(ot.tprod(A, B), ot.tprod(B, A)) > 0.1


def test_conjugate_transpose(rng):
    p = 5
    A, B = rand_q(rng, p, 3, 4), rand_q(rng, p, 4, 2)
    lhs = ot.tconjT(ot.tprod(A, B))
    rhs = ot.tprod(ot.tconjT(B), ot.tconjT(A))
    assert ot.rel_frob(lhs, rhs) < 1e-13
    # bcirc(A^H) is the quaternion conjugate transpose of bcirc(A)
    np.testing.assert_array_equal(ot.bcirc(ot.tconjT(A)), oq.qconjT(ot.bcirc(A)))
    np.testing.assert_array_equal(ot.tconjT(ot.tconjT(A)), A)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 8, 12])
def test_chi_lift_fft_route(rng, p):
    """chi commutes with bcirc, so chi(A * B) = chi(A) *_C chi(B) (complex
    T-product computed by Algorithm 2.1 with numpy's FFT)."""
    m, n, s = 3, 4, 2
    A, B = rand_q(rng, p, m, n), rand_q(rng, p, n, s)
    Cc = complex_tprod_fft(chi(A), chi(B))
    assert ot.rel_frob(ot.tprod(A, B), unchi(Cc, m, s)) < 1e-13


@pytest.mark.parametrize("p", [1, 3, 8, 10])
def test_real_case_is_algorithm_2_1(rng, p):
    """Real tensors (b = c = d = 0): T-product of Algorithm 2.1 (Prop. 2.1)."""
    A = np.zeros((4, p, 3, 5)); A[0] = rng.standard_normal((p, 3, 5))
    B = np.zeros((4, p, 5, 2)); B[0] = rng.standard_normal((p, 5, 2))
    ref = np.fft.ifft(np.fft.fft(A[0], axis=0) @ np.fft.fft(B[0], axis=0), axis=0)
    C = ot.tprod(A, B)
    np.testing.assert_allclose(C[0], ref.real, atol=1e-12)
    assert np.all(C[1:] == 0.0)


# ---------------------------------------------------------------------------
# Fourier-domain forms: the paper's coupled form agrees, the naive one does not
# ---------------------------------------------------------------------------

def fourier_paper_convention(A, B):
    """The paper's convention of the same product: the transform of conj X
    (Theorem 4.4; the quaternion conjugate of X1 + X2 j is conj X1 - X2 j),
    faces paired as i and p + 2 - i (1-based) in eqs. TC and TC2 of Remark
    5.1, and the inverse transform of conj C^.  With 0-based f the partner
    face p + 2 - i is -f mod p.  All faces at once."""
    A1, A2 = cd_planes(A)
    B1, B2 = cd_planes(B)
    F = lambda X: np.fft.fft(X, axis=0)
    a1, a2 = F(np.conj(A1)), -F(A2)
    b1, b2 = F(np.conj(B1)), -F(B2)
    r = (-np.arange(A.shape[1])) % A.shape[1]
    c1 = a1[r] @ b1[r] - np.conj(a2) @ b2[r]
    c2 = np.conj(a1[r]) @ b2 + a2 @ b1
    # conj of (c1 + c2 j) is conj c1 - c2 j
    return from_cd(np.fft.ifft(np.conj(c1), axis=0), -np.fft.ifft(c2, axis=0))


def fourier_naive(A, B):
    """Same, but every frequency treated on its own (no -f coupling)."""
    A1, A2 = cd_planes(A)
    B1, B2 = cd_planes(B)
    F = lambda X: np.fft.fft(X, axis=0)
    a1, a2, b1, b2 = F(A1), F(A2), F(B1), F(B2)
    c1 = a1 @ b1 - a2 @ np.conj(b2)
    c2 = a1 @ b2 + a2 @ np.conj(b1)
    return from_cd(np.fft.ifft(c1, axis=0), np.fft.ifft(c2, axis=0))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 8, 12, 13])
def test_coupled_fourier_forms_match_definition(rng, p):
    """The plain-DFT coupled form (oracle.tprod_fft) and the paper's own
    convention (conj-transform, faces i and p + 2 - i) both give the
    definitional product."""
    A, B = rand_q(rng, p, 4, 3), rand_q(rng, p, 3, 5)
    ref = ot.tprod(A, B)
    assert ot.rel_frob(fourier_paper_convention(A, B), ref) < 1e-13
    assert ot.rel_frob(oracle.tprod_fft(A, B), ref) < 1e-13


@pytest.mark.parametrize("mns,p", [((10, 10, 10), 50), ((6, 5, 4), 200)])
def test_algorithm_5_1_within_table_2_error(rng, mns, p):
    """Table 2 reports relative errors of at most about 2e-16 between
    Algorithm 5.1 and the definition; FP64 rounding of both routes stays
    far below 1e-14 at these sizes."""
    m, n, s = mns
    A, B = rand_q(rng, p, m, n), rand_q(rng, p, n, s)
    assert ot.rel_frob(oracle.tprod_fft(A, B), ot.tprod(A, B)) < 1e-14


@pytest.mark.parametrize("p", [3, 4, 7, 8, 16])
def test_naive_fourier_form_is_wrong(rng, p):
    """Section 3 / Example 3.1: the DFT alone does not diagonalise bcirc of a
    quaternion tensor, so dropping the -f coupling gives O(1) errors."""
    A, B = rand_q(rng, p, 4, 3), rand_q(rng, p, 3, 5)
    assert ot.rel_frob(fourier_naive(A, B), ot.tprod(A, B)) > 0.3


@pytest.mark.parametrize("p", [1, 2])
def test_naive_fourier_form_exact_for_p_le_2(rng, p):
    """For p <= 2 every frequency is its own negative, so both forms agree."""
    A, B = rand_q(rng, p, 4, 3), rand_q(rng, p, 3, 5)
    assert ot.rel_frob(fourier_naive(A, B), ot.tprod(A, B)) < 1e-13


def test_naive_fourier_form_exact_for_even_tubes(rng):
    """If every tube of B satisfies B_k = B_{-k}, its spectrum is even and the
    coupling is invisible."""
    p = 6
    A = rand_q(rng, p, 3, 3)
    B = rand_q(rng, p, 3, 2)
    B = 0.5 * (B + B[:, (-np.arange(p)) % p])
    assert ot.rel_frob(fourier_naive(A, B), ot.tprod(A, B)) < 1e-13


def test_worked_example_F4():
    """eq. (F4): F_4 circ(j, 2j, 3j, 4j) F_4^* is not diagonal."""
    rows = []
    with open(os.path.join(GOLDEN, "f4_example.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                r, c, mod = line.split()
                rows.append((int(r) - 1, int(c) - 1, float(mod)))
    p = 4
    w = np.exp(-2j * np.pi / p)                      # omega of the DFT matrix F_p
    F = np.array([[w ** (a * b) for b in range(p)] for a in range(p)]) / np.sqrt(p)
    Fq = np.stack([F.real, F.imag, np.zeros_like(F.real), np.zeros_like(F.real)])
    A = np.zeros((4, p, p))
    gen = [1.0, 2.0, 3.0, 4.0]
    for r in range(p):
        for c in range(p):
            A[2, r, c] = gen[(r - c) % p]            # circ(a1..ap): first column a1..ap
    Z = p * oq.qmatmul(oq.qmatmul(Fq, A), oq.qconjT(Fq))   # un-normalised DFT
    nz = {(r, c) for r, c, _ in rows}
    for r in range(p):
        for c in range(p):
            mod = np.sqrt(np.sum(Z[:, r, c] ** 2))
            if (r, c) in nz:
                want = [m for rr, cc, m in rows if (rr, cc) == (r, c)][0]
                assert abs(mod - want) < 1e-12
                assert abs(Z[0, r, c]) < 1e-12 and abs(Z[1, r, c]) < 1e-12
            else:
                assert mod < 1e-12
    # the same pattern i + j = 2 (mod p) in 1-based indices
    assert all(((r + 1) + (c + 1)) % p == 2 % p for r, c, _ in rows)


# ---------------------------------------------------------------------------
# Loss and adjoints
# ---------------------------------------------------------------------------

def test_adjoints_against_central_differences(rng):
    p, m, n, s = 4, 3, 2, 3
    A, B, T = rand_q(rng, p, m, n), rand_q(rng, p, n, s), rand_q(rng, p, m, s)
    G = ot.tprod(A, B) - T
    dA, dB = ot.adjoints(A, B, G)
    h = 1e-3
    for X, dX, which in [(A, dA, 0), (B, dB, 1)]:
        fd = np.zeros_like(X)
        for idx in np.ndindex(X.shape):
            Xp = X.copy(); Xp[idx] += h
            Xm = X.copy(); Xm[idx] -= h
            if which == 0:
                lp, lm = ot.loss(Xp, B, T), ot.loss(Xm, B, T)
            else:
                lp, lm = ot.loss(A, Xp, T), ot.loss(A, Xm, T)
            fd[idx] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(dX, fd, rtol=1e-8, atol=1e-9)


def test_adjoint_dot_identity(rng):
    p = 5
    A, B, Z = rand_q(rng, p, 3, 4), rand_q(rng, p, 4, 2), rand_q(rng, p, 3, 2)
    ip = lambda X, Y: float(np.sum(X * Y))
    lhs = ip(ot.tprod(A, B), Z)
    dA, dB = ot.adjoints(A, B, Z)
    assert abs(lhs - ip(A, dA)) < 1e-12 * max(1.0, abs(lhs))
    assert abs(lhs - ip(B, dB)) < 1e-12 * max(1.0, abs(lhs))


# ---------------------------------------------------------------------------
# Error measure: relative Frobenius norm over all four components
# ---------------------------------------------------------------------------

def _rel_frob_pins_hold():
    ok = True
    ones = np.ones((4, 2, 3, 3))
    ok &= abs(ot.rel_frob(ones, 2.0 * ones) - 0.5) < 1e-15
    ref = np.zeros((4, 2, 2, 2))
    ref[0, 0, 0, 0] = 3.0
    ref[3, 1, 1, 1] = 4.0
    E = np.zeros_like(ref)
    E[1, 1, 0, 1] = 1.0
    E[2, 1, 0, 1] = 2.0
    E[3, 1, 0, 1] = 2.0
    ok &= abs(ot.rel_frob(ref + E, ref) - 0.6) < 1e-15
    # an error confined to one component still counts: 1 / 5 from plane 3 alone
    E3 = np.zeros_like(ref)
    E3[3, 0, 1, 0] = 1.0
    ok &= abs(ot.rel_frob(ref + E3, ref) - 0.2) < 1e-15
    ok &= ot.rel_frob(ref, ref) == 0.0
    return bool(ok)


def test_rel_frob_hand_values():
    """||X - ref||_F / ||ref||_F, both norms over all four components: values
    worked out by hand (1/2, 3/5, 1/5 and 0)."""
    assert _rel_frob_pins_hold()


def test_rel_frob_scale_invariant_and_symmetric_in_sign(rng):
    X = rand_q(rng, 3, 4, 5)
    ref = rand_q(rng, 3, 4, 5)
    e = ot.rel_frob(X, ref)
    assert abs(ot.rel_frob(7.0 * X, 7.0 * ref) - e) < 1e-14
    assert abs(ot.rel_frob(2.0 * ref - X, ref) - e) < 1e-14      # error -E has the same norm


# ---------------------------------------------------------------------------
# Planted mistakes: the pins above must reject each of them
# ---------------------------------------------------------------------------

def _pins_hold(rng):
    p, m, n, s = 3, 2, 3, 2
    A, B = rand_q(rng, p, m, n), rand_q(rng, p, n, s)
    ok = np.allclose(ot.tprod(A, B), brute_tprod(A, B), atol=1e-12)
    ok &= np.allclose(ot.tprod_faces(A, B), brute_tprod(A, B), atol=1e-12)
    C = ot.tprod(A, B)
    ok &= ot.rel_frob(ot.tconjT(C), ot.tprod(ot.tconjT(B), ot.tconjT(A))) < 1e-12
    Z = rand_q(rng, p, m, s)
    dA, dB = ot.adjoints(A, B, Z)
    lhs = float(np.sum(C * Z))
    ok &= abs(lhs - float(np.sum(A * dA))) < 1e-10 and abs(lhs - float(np.sum(B * dB))) < 1e-10
    ok &= _rel_frob_pins_hold()
    return bool(ok)


def _mut_qmatmul_sign(X, Y):
    Z = oq.qmatmul(X, Y)
    a1, b1, c1, d1 = X
    a2, b2, c2, d2 = Y
    Z[3] = Z[3] + 2 * np.matmul(c1, b2)             # "- c1 b2" typed as "+ c1 b2"
    return Z


def _mut_qmatmul_dropped(X, Y):
    Z = oq.qmatmul(X, Y)
    Z[1] = Z[1] - np.matmul(X[2], Y[3])             # term c1 d2 dropped
    return Z


def _mut_qmatmul_swapped(X, Y):
    # operands multiplied in the wrong order (quaternions do not commute)
    a1, b1, c1, d1 = X
    a2, b2, c2, d2 = Y
    mm = np.matmul
    return np.stack([
        mm(a1, a2) - mm(b1, b2) - mm(c1, c2) - mm(d1, d2),
        mm(a1, b2) + mm(b1, a2) - mm(c1, d2) + mm(d1, c2),
        mm(a1, c2) + mm(b1, d2) + mm(c1, a2) - mm(d1, b2),
        mm(a1, d2) - mm(b1, c2) + mm(c1, b2) + mm(d1, a2),
    ])


def _mut_bcirc_index(A):
    A = np.asarray(A, dtype=np.float64)
    _, p, m, n = A.shape
    M = np.empty((4, m * p, n * p))
    for k in range(p):
        for r in range(p):
            M[:, k * m:(k + 1) * m, r * n:(r + 1) * n] = A[:, (k + r) % p]
    return M


def _mut_tconjT_no_reverse(X):
    return oq.qconjT(np.asarray(X, dtype=np.float64))


def _mut_rel_frob_squared(X, ref):
    # ||X - ref||^2 / ||ref||^2: a 1e-5 gate would then admit errors near 3e-3
    X, ref = np.asarray(X, np.float64), np.asarray(ref, np.float64)
    return float(oq.qnorm2(X - ref) / oq.qnorm2(ref))


def _mut_rel_frob_no_denominator(X, ref):
    X, ref = np.asarray(X, np.float64), np.asarray(ref, np.float64)
    return float(np.sqrt(oq.qnorm2(X - ref)))


def _mut_rel_frob_first_component(X, ref):
    # only the real component a is compared
    X, ref = np.asarray(X, np.float64), np.asarray(ref, np.float64)
    return float(np.linalg.norm(X[0] - ref[0]) / np.linalg.norm(ref[0]))


def _mut_rel_frob_max_abs(X, ref):
    X, ref = np.asarray(X, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(X - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("target,mutant", [
    ("qmatmul", _mut_qmatmul_sign),
    ("qmatmul", _mut_qmatmul_dropped),
    ("qmatmul", _mut_qmatmul_swapped),
    ("bcirc", _mut_bcirc_index),
    ("tconjT", _mut_tconjT_no_reverse),
    ("rel_frob", _mut_rel_frob_squared),
    ("rel_frob", _mut_rel_frob_no_denominator),
    ("rel_frob", _mut_rel_frob_first_component),
    ("rel_frob", _mut_rel_frob_max_abs),
])
def test_planted_mistakes_are_caught(rng, monkeypatch, target, mutant):
    assert _pins_hold(rng)
    monkeypatch.setattr(ot, target, mutant)
    assert not _pins_hold(rng)
