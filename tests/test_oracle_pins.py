"""Pins of the FP64 oracle against facts fixed by mathematics, not by itself.

The paper prints no worked numeric example of a product, so each oracle
function is pinned by: integer-exact inputs (exact in binary64, so the
result is the exact integer product), closed forms (identity, permutation,
rank-1, orthonormal bases), exact rational brute force of tiny cases,
exhaustive {-1,0,1} 2x2 cases, compensated dot products at full size and the
associativity of the low-rank chain.  Each pin is chosen so that a dropped
term, a wrong sign, a wrong index or a transposed operand fails it.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

from paper_2311_07602_amd import inputs

U64 = 2.0 ** -53


def gamma(n):
    return n * U64 / (1 - n * U64)


def exact_int_matmul(X, Y):
    """Exact product of integer-valued float matrices via Python ints."""
    Xi = X.astype(np.int64); Yi = Y.astype(np.int64)
    return (Xi @ Yi).astype(np.float64)


# ---------------------------------------------------------------- DENSE_TS

@pytest.mark.parametrize("b,r", [(7, 3), (64, 16), (33, 5)])
def test_dense_ts_identity_and_permutation(orc, b, r):
    rng = np.random.default_rng(1)
    U = inputs.normal_f(rng, b, r)
    C = orc.dense_ts([np.asfortranarray(np.eye(b))], [U])[0]
    assert np.array_equal(C, U)
    perm = rng.permutation(b)
    P = np.asfortranarray(np.eye(b)[perm])
    C = orc.dense_ts([P], [U])[0]
    assert np.array_equal(C, U[perm])


def test_dense_ts_rank1_integer(orc):
    rng = np.random.default_rng(2)
    x = rng.integers(-8, 9, size=(40, 1)).astype(float)
    y = rng.integers(-8, 9, size=(40, 1)).astype(float)
    A = np.asfortranarray(x @ y.T)
    U = inputs.integer_f(rng, 40, 6)
    C = orc.dense_ts([A], [U])[0]
    assert np.array_equal(C, x @ (y.T @ U))


def test_dense_ts_integer_exact_nonsquare_ld(orc):
    rng = np.random.default_rng(3)
    m, k, n = 19, 23, 7
    A = orc.col_major(m, k, ld=m + 5); A[...] = inputs.integer_f(rng, m, k)
    U = orc.col_major(k, n, ld=k + 3); U[...] = inputs.integer_f(rng, k, n)
    Cbuf = np.full((n, m + 2), -7.0)
    C = Cbuf.T[:m, :n]
    orc.dense_ts([A], [U], out=[C])
    assert np.array_equal(C, exact_int_matmul(np.asarray(A), np.asarray(U)))
    assert np.all(Cbuf.T[m:, :] == -7.0), "oracle wrote into the leading-dimension gap"


# ---------------------------------------------------------------- INNER

def test_inner_unit_vectors(orc):
    b, r = 50, 8
    E = np.asfortranarray(np.eye(b)[:, :r])
    T = orc.inner([E], [E])[0]
    assert np.array_equal(T, np.eye(r))


def test_inner_permuted_identity_columns(orc):
    rng = np.random.default_rng(4)
    b, r = 40, 6
    pi = rng.permutation(b)[:r]
    E = np.asfortranarray(np.eye(b)[:, pi])
    U2 = inputs.normal_f(rng, b, r)
    T = orc.inner([E], [U2])[0]
    assert np.array_equal(T, U2[pi, :])


def test_inner_integer_exact(orc):
    rng = np.random.default_rng(5)
    b, m, n = 77, 9, 5
    V1 = inputs.integer_f(rng, b, m); U2 = inputs.integer_f(rng, b, n)
    T = orc.inner([V1], [U2])[0]
    assert np.array_equal(T, exact_int_matmul(V1.T, U2))


def test_inner_orthonormal_gives_sigma(orc):
    rng = np.random.default_rng(6)
    b, r = 256, 16
    Q = inputs.orthonormal_f(rng, b, r)
    sig = inputs.sigma_profile(r)
    V1 = np.asfortranarray(Q * sig[None, :])
    T = orc.inner([V1], [Q])[0]
    D = orc.inner([np.abs(V1)], [np.abs(Q)])[0]
    # Q^T Q = I up to the QR's own rounding (~1e-15); diag(sigma) Q^T Q
    assert np.all(np.abs(T - np.diag(sig)) <= 1e-13 * np.maximum(D, 1e-300) + 1e-14 * sig[:, None])


# ---------------------------------------------------------------- RECOMP

def test_recomp_single_core_entry_is_outer_product(orc):
    rng = np.random.default_rng(7)
    b, r = 30, 5
    U1 = inputs.normal_f(rng, b, r); V2 = inputs.normal_f(rng, 21, r)
    S = np.zeros((r, r), order="F"); S[0, 0] = 1.0
    W = orc.recomp([U1], [S], [V2])[0]
    assert np.array_equal(W, np.outer(U1[:, 0], V2[:, 0]))


def test_recomp_identity_core_unit_bases(orc):
    b, r = 24, 6
    E = np.asfortranarray(np.eye(b)[:, :r])
    W = orc.recomp([E], [np.asfortranarray(np.eye(r))], [E])[0]
    expect = np.zeros((b, b)); expect[:r, :r] = np.eye(r)
    assert np.array_equal(W, expect)


def test_recomp_integer_exact_association(orc):
    rng = np.random.default_rng(8)
    m, n, k = 17, 13, 6
    U1 = inputs.integer_f(rng, m, k); S = inputs.integer_f(rng, k, k); V2 = inputs.integer_f(rng, n, k)
    W = orc.recomp([U1], [S], [V2])[0]
    assert np.array_equal(W, exact_int_matmul(U1, exact_int_matmul(S, V2.T)))


def test_recomp_singular_values(orc):
    rng = np.random.default_rng(9)
    b, r = 64, 8
    U1 = inputs.orthonormal_f(rng, b, r); V2 = inputs.orthonormal_f(rng, b, r)
    sig = inputs.sigma_profile(r, -4.0)
    W = orc.recomp([U1], [np.asfortranarray(np.diag(sig))], [V2])[0]
    sv = np.linalg.svd(W, compute_uv=False)[:r]
    assert np.allclose(sv, sig, rtol=1e-10, atol=1e-14)
    assert np.all(np.linalg.svd(W, compute_uv=False)[r:] < 1e-14)


# ------------------------------------------------------------ chain / Alg. 1

def test_chain_associativity(orc):
    """U1 (V1^T U2) V2^T equals the explicitly formed (U1 V1^T)(U2 V2^T)."""
    ci = inputs.chain_instance(2, 0, 128, 16)
    T, W = orc.chain([ci.V1], [ci.U2], [ci.U1], [ci.V2])
    A1 = orc.dense_ts([ci.U1], [np.asfortranarray(ci.V1.T)])[0]          # U1 V1^T  (b x b)
    B2 = orc.dense_ts([ci.U2], [np.asfortranarray(ci.V2.T)])[0]          # U2 V2^T
    dense = orc.dense_ts([A1], [B2])[0]
    aU1, aV1, aU2, aV2 = (np.abs(x) for x in (ci.U1, ci.V1, ci.U2, ci.V2))
    Tabs = orc.inner([aV1], [aU2])[0]
    D = orc.recomp([np.asfortranarray(aU1)], [Tabs], [np.asfortranarray(aV2)])[0]
    b, r = 128, 16
    # Each evaluation is within (gamma_b + 2 gamma_r) D of the exact product
    # (the dense one also within that order), so they differ by at most twice it.
    W = W[0]
    assert np.all(np.abs(W - dense) <= 2 * (gamma(b) + 2 * gamma(r)) * D)
    # a dropped or wrong term would be of the size of D itself
    assert np.max(np.abs(W - dense) / D) < 1e-13


def test_lr_mult_matches_six_loop_form_integer(orc):
    """Alg. 1 (three products) equals the paper's six nested loops (Alg. 2),
    which accumulate G directly; on integer inputs both are exact."""
    rng = np.random.default_rng(10)
    kk, ra, rb = 12, 3, 4
    AV = inputs.integer_f(rng, kk, ra); BU = inputs.integer_f(rng, kk, rb)
    AX = inputs.integer_f(rng, ra, ra); BX = inputs.integer_f(rng, rb, rb)
    G = orc.lr_mult([AV], [BU], [AX], [BX])[0]
    G6 = [[0] * rb for _ in range(ra)]
    for m in range(ra):                       # loop 2
        for n in range(rb):                   # loop 3
            cmn = 0
            for k in range(kk):               # loop 4
                cmn += int(AV[k, m]) * int(BU[k, n])
            for x in range(ra):               # loop 5
                exn = int(AX[x, m]) * cmn
                for y in range(rb):           # loop 6
                    G6[x][y] += exn * int(BX[n, y])
    assert np.array_equal(G, np.array(G6, dtype=np.float64))


# ------------------------------------------------------ exact brute force

def _exact_product(X, Y):
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    Yf = [[Fraction(float(v)) for v in row] for row in Y]
    return [[sum(Xf[i][l] * Yf[l][j] for l in range(len(Yf))) for j in range(len(Yf[0]))]
            for i in range(len(Xf))]


@pytest.mark.parametrize("m,k,n", [(4, 4, 4), (4, 2, 4), (2, 4, 2), (4, 4, 2)])
def test_bruteforce_rational(orc, m, k, n):
    rng = np.random.default_rng(11 + m + 3 * k + 7 * n)
    for trial in range(20):
        A = inputs.normal_f(rng, m, k); U = inputs.normal_f(rng, k, n)
        ex = _exact_product(A, U)
        D = np.abs(A) @ np.abs(U)
        C = orc.dense_ts([A], [U])[0]
        T = orc.inner([np.asfortranarray(A.T)], [U])[0]
        for i in range(m):
            for j in range(n):
                e = Fraction(float(C[i, j])) - ex[i][j]
                assert abs(float(e)) <= gamma(k) * D[i, j]
                assert float(T[i, j]) == float(C[i, j])   # same sum, same order


def test_exhaustive_pm1_2x2(orc):
    vals = (-1.0, 0.0, 1.0)
    As, Us = [], []
    for a in itertools.product(vals, repeat=4):
        for u in itertools.product(vals, repeat=4):
            As.append(np.asfortranarray(np.array(a).reshape(2, 2)))
            Us.append(np.asfortranarray(np.array(u).reshape(2, 2)))
    Cs = orc.dense_ts(As, Us)
    Ts = orc.inner(As, Us)
    for A, U, C, T in zip(As, Us, Cs, Ts):
        assert np.array_equal(C, A @ U)
        assert np.array_equal(T, A.T @ U)
    assert len(As) == 6561


def test_recomp_rational_small(orc):
    rng = np.random.default_rng(12)
    for trial in range(10):
        U1 = inputs.normal_f(rng, 4, 3); S = inputs.normal_f(rng, 3, 3); V2 = inputs.normal_f(rng, 4, 3)
        W = orc.recomp([U1], [S], [V2])[0]
        ex = _exact_product(U1, _exact_product(S, V2.T))
        D = np.abs(U1) @ (np.abs(S) @ np.abs(V2).T)
        for i in range(4):
            for j in range(4):
                assert abs(float(Fraction(float(W[i, j])) - ex[i][j])) <= 2 * gamma(3) * D[i, j]


# ----------------------------------------------------------- at full size

def test_dot2_and_library_at_size(orc):
    """Sampled entries of a full-size product against the compensated Dot2
    (accurate to about u^2 k) and against numpy's BLAS product."""
    b, r = 1024, 32
    A, U = inputs.dense_ts_instance(3, 0, b, r)
    C = orc.dense_ts([A], [U])[0]
    D = orc.dense_ts([np.abs(A)], [np.abs(U)])[0]
    rng = np.random.default_rng(13)
    for _ in range(64):
        i, j = int(rng.integers(b)), int(rng.integers(r))
        ref = orc.dot2(np.ascontiguousarray(A[i, :]), np.ascontiguousarray(U[:, j]))
        assert abs(C[i, j] - ref) <= gamma(b) * D[i, j]
        assert abs(C[i, j] - ref) <= 1e-14 * D[i, j]          # typical error
    Cnp = A @ U
    assert np.all(np.abs(C - Cnp) <= 2 * gamma(b) * D)


def test_zero_sizes(orc):
    A = np.zeros((3, 0), order="F"); U = np.zeros((0, 2), order="F")
    C = orc.dense_ts([A], [U])[0]
    assert C.shape == (3, 2) and np.all(C == 0)
    V = np.zeros((0, 3), order="F")
    T = orc.inner([V], [np.zeros((0, 4), order="F")])[0]
    assert T.shape == (3, 4) and np.all(T == 0)
    W = orc.recomp([np.zeros((5, 0), order="F")], [np.zeros((0, 0), order="F")], [np.zeros((6, 0), order="F")])[0]
    assert W.shape == (5, 6) and np.all(W == 0)


def test_thread_count_invariance(orc):
    As, Us = [], []
    for i in range(16):
        A, U = inputs.dense_ts_instance(1, i, 64, 16)
        As.append(A); Us.append(U)
    C1 = orc.dense_ts(As, Us, nthreads=1)
    C8 = orc.dense_ts(As, Us, nthreads=8)
    for a, b in zip(C1, C8):
        assert np.array_equal(a, b)


def test_error_metric(orc):
    C = np.array([[1.0, 0.0], [2.0, 3.0]]); R = np.array([[1.0, 0.0], [2.0 + 1e-10, 3.0]])
    D = np.array([[1.0, 0.0], [10.0, 1.0]])
    assert orc.normalized_error(C, R, D) == pytest.approx(1e-11, rel=1e-3)
    C2 = C.copy(); C2[0, 1] = 1e-300
    assert orc.normalized_error(C2, R, D) == float("inf")
    C3 = C.copy(); C3[0, 1] = -0.0
    assert orc.normalized_error(C3, R, D) == pytest.approx(1e-11, rel=1e-3)
    C4 = C.copy(); C4[1, 1] = np.nan
    assert orc.normalized_error(C4, R, D) == float("inf")


def test_normwise_error_hand_computed(orc):
    """max_ij |C - Cref| / (||A||_F ||B||_F) on values worked by hand:
    A = [[3, 0], [0, 4]] (||A||_F = 5), B = [[1, 2], [2, 4]] (||B||_F = 5);
    the largest entry of |C - Cref| is 0.5, so the error is 0.5 / 25."""
    A = np.array([[3.0, 0.0], [0.0, 4.0]]); B = np.array([[1.0, 2.0], [2.0, 4.0]])
    Cref = A @ B
    C = Cref.copy(); C[0, 1] -= 0.5; C[1, 0] += 0.25
    a_fro, b_fro = float(np.sqrt((A * A).sum())), float(np.sqrt((B * B).sum()))
    assert (a_fro, b_fro) == (5.0, 5.0)
    assert orc.normwise_error(C, Cref, a_fro, b_fro) == 0.02
    assert orc.normwise_error(Cref, Cref, a_fro, b_fro) == 0.0
    assert orc.normwise_error(np.zeros((0, 3)), np.zeros((0, 3)), 1.0, 1.0) == 0.0
    # zero operands: an exact zero result has no error, anything else is unbounded
    assert orc.normwise_error(np.zeros((2, 2)), np.zeros((2, 2)), 0.0, 5.0) == 0.0
    assert orc.normwise_error(C, Cref, 0.0, 5.0) == float("inf")


def test_dot2_ill_conditioned_exact(orc):
    """Dot2 recovers sums that plain summation loses entirely: the rounding
    error of a product (a*a - fl(a*a)) and cancellation of huge terms.  The
    exact values are computed with rationals."""
    rng = np.random.default_rng(14)
    for _ in range(50):
        a = float(rng.standard_normal()) * 3.0
        p = a * a
        x = np.array([a, 1.0]); y = np.array([a, -p])
        ex = Fraction(a) * Fraction(a) - Fraction(p)
        assert ex != 0 or a == 0
        assert orc.dot2(x, y) == float(ex)
        big = float(rng.integers(1, 1000)) * 2.0 ** 60
        small = float(rng.standard_normal())
        x = np.array([big, small, -big]); y = np.ones(3)
        assert orc.dot2(x, y) == small


# ------------------------------------------------------ BLR matrix x RHS

def _blr_host(rng, nb, b, r, nrhs, f):
    D = [f(rng, b, b) for _ in range(nb)]
    U = [[None if i == j else f(rng, b, r) for j in range(nb)] for i in range(nb)]
    V = [[None if i == j else f(rng, b, r) for j in range(nb)] for i in range(nb)]
    X = [f(rng, b, nrhs) for _ in range(nb)]
    return D, U, V, X


def _assembled(D, U, V):
    nb, b = len(D), D[0].shape[0]
    A = np.zeros((nb * b, nb * b))
    for i in range(nb):
        for j in range(nb):
            A[i * b:(i + 1) * b, j * b:(j + 1) * b] = D[i] if i == j else U[i][j] @ V[i][j].T
    return A


@pytest.mark.parametrize("nb,b,r,nrhs", [(3, 5, 2, 4), (4, 8, 3, 1), (1, 6, 2, 3), (5, 7, 1, 2)])
def test_blr_matvec_equals_assembled_product_integer(orc, nb, b, r, nrhs):
    """On integer blocks every partial sum is exact, so the BLR evaluation
    U_ij (V_ij^T X_j) must equal the assembled dense matrix times X exactly
    (numpy's product of the assembled matrix, not the oracle's loops)."""
    rng = np.random.default_rng(20 + nb + b)
    D, U, V, X = _blr_host(rng, nb, b, r, nrhs, inputs.integer_f)
    Y = np.vstack(orc.blr_matvec(D, U, V, X))
    assert np.array_equal(Y, _assembled(D, U, V) @ np.vstack(X))


def test_blr_matvec_within_bound_of_assembled_product(orc):
    """N(0,1) blocks: the two evaluation orders differ only by rounding,
    within gamma_n of the sum of absolute terms."""
    rng = np.random.default_rng(31)
    nb, b, r, nrhs = 4, 16, 3, 2
    D, U, V, X = _blr_host(rng, nb, b, r, nrhs, inputs.normal_f)
    Y = np.vstack(orc.blr_matvec(D, U, V, X))
    Yd = _assembled(D, U, V) @ np.vstack(X)
    ab = lambda m: None if m is None else np.asfortranarray(np.abs(m))
    Dabs = np.vstack(orc.blr_matvec([ab(d) for d in D], [[ab(u) for u in row] for row in U],
                                    [[ab(v) for v in row] for row in V], [ab(x) for x in X]))
    n = nb * b + r
    assert np.all(np.abs(Y - Yd) <= 2 * gamma(n) * Dabs)
    assert np.max(np.abs(Y - Yd) / Dabs) < 1e-14


# ------------------------------------------ recompressed low-rank product

def test_lr_mult_round_recovers_a_planted_spectrum(orc):
    """A core with known singular values: A_X = P diag(s) Q^T with A_V^T B_U
    = I and B_X = I (orthonormal P, Q); the recompressed product keeps exactly
    the singular values above tol * s_1, in order, and U diag(sigma) V^T is
    the truncated product."""
    rng = np.random.default_rng(41)
    b, r = 40, 6
    s = np.array([3.0, 2.0, 1.0, 1e-3, 1e-9, 1e-14])
    P = inputs.orthonormal_f(rng, r, r); Q = inputs.orthonormal_f(rng, r, r)
    AX = np.asfortranarray(P @ np.diag(s) @ Q.T)
    W = inputs.orthonormal_f(rng, b, r)                 # A_V = B_U = W: A_V^T B_U = I
    AU = inputs.orthonormal_f(rng, b, r); BV = inputs.orthonormal_f(rng, b, r)
    BX = np.asfortranarray(np.eye(r))
    for tol, kmax, want in ((1e-6, 6, 4), (1e-12, 6, 5), (0.0, 3, 3), (0.9, 6, 1)):
        U, sig, V, k = orc.lr_mult_round(AU, W, AX, W, BX, BV, kmax, tol)
        assert k == want
        assert np.allclose(sig[:k], s[:k], rtol=1e-13, atol=1e-15)
        assert np.all(sig[k:] == 0) and np.all(U[:, k:] == 0) and np.all(V[:, k:] == 0)
        full = AU @ AX @ BV.T                            # the exact product (A_V^T B_U = I)
        trunc = AU @ P[:, :k] @ np.diag(s[:k]) @ Q[:, :k].T @ BV.T
        got = U[:, :k] @ np.diag(sig[:k]) @ V[:, :k].T
        assert np.max(np.abs(got - trunc)) < 1e-13
        assert np.max(np.abs(got - full)) <= (s[k] if k < r else 0) + 1e-13
        assert np.allclose(U[:, :k].T @ U[:, :k], np.eye(k), atol=1e-13)


def test_blr_matvec_selected_rows_equal_full_evaluation(orc):
    rng = np.random.default_rng(32)
    D, U, V, X = _blr_host(rng, 5, 6, 2, 3, inputs.normal_f)
    full = orc.blr_matvec(D, U, V, X)
    part = orc.blr_matvec(D, U, V, X, rows=[3, 0])
    assert np.array_equal(part[0], full[3]) and np.array_equal(part[1], full[0])


# ----------------------------------------------------- Householder QR

def _qr_checks(W, Q, R, tol=1e-14):
    m, n = W.shape
    p = min(m, n)
    assert Q.shape == (m, p) and R.shape == (p, n)
    scale = max(np.abs(W).max(), 1e-300)
    assert np.max(np.abs(Q @ R - W)) <= tol * (m + n) * scale
    assert np.max(np.abs(Q.T @ Q - np.eye(p))) <= tol * (m + n)
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R) >= 0)


def test_householder_qr_hadamard_closed_form(orc):
    """Columns of a Hadamard matrix are orthogonal with norm 2: every
    reflector's quantities are exact in binary64, so R = 2 I and Q = H / 2
    bit for bit (H_0's sign case x0 > 0 and the later x0 <= 0 cases both
    occur)."""
    H = np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], dtype=float)
    (Q, R), = orc.householder_qr([np.asfortranarray(H)])
    assert np.array_equal(R, 2.0 * np.eye(4))
    assert np.array_equal(Q, H / 2.0)
    # a signed column permutation (the first pivot negative, so the x0 <= 0
    # branch starts): R = 2 I and Q = Hs / 2 to rounding (thirds appear)
    Hs = np.asfortranarray(H[:, [2, 0, 3, 1]] * np.array([-1.0, 1.0, -1.0, 1.0]))
    (Q2, R2), = orc.householder_qr([Hs])
    assert np.max(np.abs(R2 - 2.0 * np.eye(4))) <= 4 * 2.0 ** -52
    assert np.max(np.abs(Q2 - Hs / 2.0)) <= 4 * 2.0 ** -52


@pytest.mark.parametrize("m,n", [(10, 4), (4, 4), (3, 6), (64, 24), (1, 1), (5, 1), (1, 5), (37, 36)])
def test_householder_qr_invariants_and_library(orc, m, n):
    """Q R = W, orthonormal Q, upper-trapezoidal R with a non-negative
    diagonal; with full column rank Q and R are unique, so they agree with
    LAPACK's QR (numpy) once its signs are normalised the same way."""
    rng = np.random.default_rng(m * 100 + n)
    W = inputs.normal_f(rng, m, n)
    (Q, R), = orc.householder_qr([W])
    _qr_checks(W, Q, R)
    q, r = np.linalg.qr(W)
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    assert np.max(np.abs(q * sg - Q)) <= 1e-13
    assert np.max(np.abs((r.T * sg).T - R)) <= 1e-13 * np.abs(W).max() * m


def test_householder_qr_ld_gap_and_batch(orc):
    rng = np.random.default_rng(5)
    Ws = []
    for m, n, ld in [(9, 3, 12), (6, 6, 7), (4, 2, 4)]:
        W = orc.col_major(m, n, ld)
        W[:, :] = rng.standard_normal((m, n))
        Ws.append(W)
    before = [W.copy() for W in Ws]
    out = orc.householder_qr(Ws)
    for W, W0, (Q, R) in zip(Ws, before, out):
        _qr_checks(W, Q, R)
        assert np.array_equal(W, W0)           # the input is read only


def test_householder_qr_gram_exact_integer(orc):
    """R^T R = W^T W: the Gram matrix of integer columns is exact in
    integers; each entry of R^T R must match it to rounding."""
    rng = np.random.default_rng(6)
    for m, n in [(7, 3), (5, 5), (12, 4)]:
        Wi = rng.integers(-3, 4, size=(m, n))
        W = np.asfortranarray(Wi.astype(float))
        (Q, R), = orc.householder_qr([W])
        G = exact_int_matmul(Wi.T, Wi)
        assert np.max(np.abs(R.T @ R - G)) <= 64 * 2.0 ** -52 * (np.abs(Wi).max() ** 2) * m


def test_householder_qr_rank_deficient_and_sign_cases(orc):
    """Duplicate and zero columns (the stacked bases of two blocks sharing a
    basis) still give Q R = W with orthonormal Q; a column that is already a
    negative multiple of e_j takes the sign flip (beta = 2) and yields a
    non-negative R_jj."""
    rng = np.random.default_rng(8)
    A = inputs.normal_f(rng, 20, 3)
    W = np.asfortranarray(np.hstack([A, A[:, [1]], np.zeros((20, 1)), A[:, [0]] * -2.0]))
    (Q, R), = orc.householder_qr([W])
    _qr_checks(W, Q, R, tol=1e-13)
    assert np.max(np.abs(np.diag(R)[3:])) <= 1e-13 * np.abs(W).max() * 20
    E = np.asfortranarray(np.array([[-3.0, 1.0], [0.0, 2.0], [0.0, 0.0]]))
    (Q, R), = orc.householder_qr([E])
    assert np.array_equal(R, np.array([[3.0, -1.0], [0.0, 2.0]]))
    assert np.array_equal(Q, np.array([[-1.0, 0.0], [0.0, 1.0], [0.0, 0.0]]))


# ------------------------------------------------- rounded addition

def _lr_blocks(rng, b, ra, rb):
    return (inputs.normal_f(rng, b, ra), inputs.normal_f(rng, b, ra), inputs.normal_f(rng, ra, ra),
            inputs.normal_f(rng, b, rb), inputs.normal_f(rng, rb, rb), inputs.normal_f(rng, b, rb))


@pytest.mark.parametrize("b,ra,rb,kmax", [(30, 4, 3, 7), (16, 5, 5, 10), (6, 4, 4, 6), (25, 1, 6, 3)])
def test_lr_add_round_equals_dense_truncated_svd(orc, b, ra, rb, kmax):
    """The rounded addition is the truncated SVD of the dense sum A + B: the
    singular values agree with LAPACK's SVD of the explicitly formed b x b
    sum, and U diag(sigma) V^T with its truncation (N(0,1) factors: the
    spectrum has gaps)."""
    rng = np.random.default_rng(b * 7 + ra + rb)
    AU, AV, AX, BU, BX, BV = _lr_blocks(rng, b, ra, rb)
    S = AU @ AX @ AV.T + BU @ BX @ BV.T
    X, s, Yt = np.linalg.svd(S)
    U, sig, V, k = orc.lr_add_round(AU, AV, AX, BU, BX, BV, kmax, 0.0)
    kk = min(kmax, ra + rb, b)
    assert k == kk
    assert np.max(np.abs(sig[:k] - s[:k])) <= 1e-12 * s[0]
    assert np.all(sig[k:] == 0) and np.all(U[:, k:] == 0) and np.all(V[:, k:] == 0)
    trunc = X[:, :k] @ np.diag(s[:k]) @ Yt[:k]
    assert np.max(np.abs(U[:, :k] @ np.diag(sig[:k]) @ V[:, :k].T - trunc)) <= 1e-11 * s[0]
    assert np.allclose(U[:, :k].T @ U[:, :k], np.eye(k), atol=1e-13)
    assert np.allclose(V[:, :k].T @ V[:, :k], np.eye(k), atol=1e-13)


def test_lr_add_round_planted_spectrum(orc):
    """A_U, B_U (and A_V, B_V) are complementary column blocks of orthonormal
    P (and Q) and the cores are diagonal: A + B = P diag(s) Q^T, so the
    singular values are the planted ones and the tolerance decides k."""
    rng = np.random.default_rng(43)
    b, ra, rb = 50, 4, 3
    s = np.array([5.0, 1e-3, 2.0, 1e-9, 3.0, 1e-14, 0.5])
    P = inputs.orthonormal_f(rng, b, ra + rb); Q = inputs.orthonormal_f(rng, b, ra + rb)
    AU, BU = np.asfortranarray(P[:, :ra]), np.asfortranarray(P[:, ra:])
    AV, BV = np.asfortranarray(Q[:, :ra]), np.asfortranarray(Q[:, ra:])
    AX, BX = np.asfortranarray(np.diag(s[:ra])), np.asfortranarray(np.diag(s[ra:]))
    order = np.argsort(-s)
    for tol, kmax, want in ((1e-6, 7, 5), (1e-12, 7, 6), (0.0, 3, 3), (0.5, 7, 2)):
        U, sig, V, k = orc.lr_add_round(AU, AV, AX, BU, BX, BV, kmax, tol)
        assert k == want
        assert np.allclose(sig[:k], s[order[:k]], rtol=1e-13, atol=1e-15)
        keep = order[:k]
        trunc = P[:, keep] @ np.diag(s[keep]) @ Q[:, keep].T
        assert np.max(np.abs(U[:, :k] @ np.diag(sig[:k]) @ V[:, :k].T - trunc)) < 1e-13


def test_lr_add_round_shared_bases_and_cancellation(orc):
    """B with the same orthonormal bases as A: the stacked bases are exactly
    rank deficient and A + B = A_U (A_X + B_X) A_V^T, whose singular values
    are those of A_X + B_X.  B = -A cancels to the zero block."""
    rng = np.random.default_rng(44)
    b, r = 40, 5
    AU = inputs.orthonormal_f(rng, b, r); AV = inputs.orthonormal_f(rng, b, r)
    AX = inputs.normal_f(rng, r, r); BX = inputs.normal_f(rng, r, r)
    U, sig, V, k = orc.lr_add_round(AU, AV, AX, AU, BX, AV, 2 * r, 1e-10)
    s = np.linalg.svd(AX + BX, compute_uv=False)
    assert k == r
    assert np.max(np.abs(sig[:r] - s)) <= 1e-13 * s[0]
    full = AU @ (AX + BX) @ AV.T
    assert np.max(np.abs(U[:, :k] @ np.diag(sig[:k]) @ V[:, :k].T - full)) <= 1e-13 * s[0]
    # B = -A: the sum is zero up to the rounding of the QR and of the core,
    # so every singular value is at the noise level of A's
    U, sig, V, k = orc.lr_add_round(AU, AV, AX, AU, np.asfortranarray(-AX), AV, 2 * r, 0.0)
    sa = np.linalg.svd(AX, compute_uv=False)[0]
    assert np.all(sig <= 16 * r * 2.0 ** -52 * sa)
    assert np.max(np.abs(U[:, :k] @ np.diag(sig[:k]) @ V[:, :k].T)) <= 16 * r * 2.0 ** -52 * sa
