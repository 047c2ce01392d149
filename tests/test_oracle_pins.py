"""Pins of the CPU oracle against facts fixed by the mathematics, not by the oracle.

Each test names what it pins and which plausible mistake it would catch:
exact rational arithmetic and pure-Python IEEE loops on tiny shapes (any wrong
index, sign, dropped term or transposed operand), identity and permutation
matrices, integer-valued inputs whose products are exact, the all-ones closed form,
the transpose identity, the componentwise error bound gamma_{k+2} (Higham,
"Accuracy and Stability of Numerical Algorithms", 2nd ed., Sec. 3.5), and the BLAS
rules for alpha == 0 / beta == 0 (the operation of the paper's Sec. 2, Eq. 1).
"""
import ctypes
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth

U64 = 2.0 ** -53


def gamma(n, u=U64):
    return n * u / (1 - n * u)


def exact_gemm(alpha, A, B, beta, C):
    """alpha*A*B + beta*C in exact rational arithmetic (Fractions of the doubles)."""
    m, k = A.shape
    n = B.shape[1]
    out = [[None] * n for _ in range(m)]
    fa, fb = Fraction(alpha), Fraction(beta)
    for i in range(m):
        for j in range(n):
            s = sum((Fraction(A[i, p]) * Fraction(B[p, j]) for p in range(k)), Fraction(0))
            out[i][j] = fa * s + (fb * Fraction(C[i, j]) if beta != 0 else 0)
    return out


def python_loop_gemm(alpha, A, B, beta, C):
    """Eq. 1 with Python floats: one IEEE binary64 rounding per +, * (no fusion)."""
    m, k = A.shape
    n = B.shape[1]
    out = np.array(C, dtype=np.float64, copy=True)
    for i in range(m):
        for j in range(n):
            acc = 0.0
            for p in range(k):
                acc = acc + float(A[i, p]) * float(B[p, j])
            out[i, j] = alpha * acc if beta == 0 else alpha * acc + beta * float(C[i, j])
    return out


TINY = [0, 1, 2, 3, 5, 7, 16, 17]


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (2, 3, 5), (3, 2, 7), (5, 7, 3),
                                   (7, 5, 16), (16, 1, 17), (1, 17, 2), (17, 16, 5)])
def test_tiny_matches_python_ieee_loop_bitwise(orc, m, n, k):
    A = synth.uniform_pm1((m, k), 11 + m)
    B = synth.uniform_pm1((k, n), 13 + n)
    C = synth.uniform_pm1((m, n), 17 + k)
    for alpha, beta in [(1.5, 0.5), (-0.75, 0.0), (1.0, 1.0), (2.0, -3.25)]:
        got = orc.gemm_f64(alpha, A, B, beta, C)
        want = python_loop_gemm(alpha, A, B, beta, C)
        assert np.array_equal(got, want), (alpha, beta)


@pytest.mark.parametrize("m,n,k", [(a, b, c) for a, b, c in itertools.product([1, 3, 7], [2, 5], [1, 16, 17])])
def test_tiny_within_gamma_of_exact_rational(orc, m, n, k):
    A = synth.uniform_pm1((m, k), 101)
    B = synth.uniform_pm1((k, n), 102)
    C = synth.uniform_pm1((m, n), 103)
    alpha, beta = 1.5, 0.5
    got = orc.gemm_f64(alpha, A, B, beta, C)
    ex = exact_gemm(alpha, A, B, beta, C)
    absAB = np.abs(A) @ np.abs(B)
    for i in range(m):
        for j in range(n):
            bound = gamma(k + 2) * (abs(alpha) * absAB[i, j] + abs(beta) * abs(C[i, j]))
            assert abs(Fraction(got[i, j]) - ex[i][j]) <= Fraction(bound) * Fraction(1 + 1e-12)


def test_dot2_matches_exact_rational_to_about_u_squared(orc):
    """Dot2's bound: |res - exact| <= u|exact| + gamma_k^2 * sum|a_p b_p| (Ogita,
    Rump, Oishi 2005, Prop. 5.5), checked on ill-conditioned rows where plain
    FP64 loses every digit."""
    k = 40
    A = synth.uniform_pm1((4, k), 7)
    B = synth.uniform_pm1((k, 3), 8)
    # Row 0 x column 0: a huge term at p = 0 absorbs the small ones in plain FP64 and
    # is cancelled at p = k-1, so plain FP64 returns a multiple of 256.
    A[0, 0], A[0, k - 1] = 2.0 ** 60, 2.0 ** 60
    B[0, 0], B[k - 1, 0] = 1.0, -1.0
    ex = exact_gemm(1.0, A, B, 0.0, np.zeros((4, 3)))
    got = orc.gemm_dot2(1.0, A, B)
    plain = orc.gemm_f64(1.0, A, B)
    absAB = np.abs(A) @ np.abs(B)
    for i in range(4):
        for j in range(3):
            bound = U64 * abs(ex[i][j]) + gamma(k) ** 2 * absAB[i, j]
            assert abs(Fraction(got[i, j]) - ex[i][j]) <= Fraction(bound)
    assert abs(float(ex[0][0])) > 1e-3
    assert abs(got[0, 0] - float(ex[0][0])) <= 4 * U64 * abs(float(ex[0][0]))
    assert abs(plain[0, 0] - float(ex[0][0])) > 0.5 * abs(float(ex[0][0]))


def test_identity_and_permutation_bitwise(orc):
    A = synth.uniform_pm1((33, 19), 1)
    I19 = np.eye(19)
    I33 = np.eye(33)
    assert np.array_equal(orc.gemm_f64(1.0, A, I19), A)
    assert np.array_equal(orc.gemm_f64(1.0, I33, A), A)
    perm = np.array([(7 * i + 3) % 33 for i in range(33)])
    P = np.zeros((33, 33))
    P[np.arange(33), perm] = 1.0     # (P A)[i] = A[perm[i]]
    assert np.array_equal(orc.gemm_f64(1.0, P, A), A[perm])
    permc = np.array([(5 * j + 2) % 19 for j in range(19)])
    Q = np.zeros((19, 19))
    Q[permc, np.arange(19)] = 1.0    # (A Q)[:, j] = A[:, permc[j]]
    assert np.array_equal(orc.gemm_f64(1.0, A, Q), A[:, permc])


@pytest.mark.parametrize("m,n,k", [(37, 29, 300), (64, 64, 64), (5, 300, 1000)])
def test_integer_valued_exact(orc, m, n, k):
    A = synth.integer_valued((m, k), 21, 8)
    B = synth.integer_valued((k, n), 22, 8)
    C = synth.integer_valued((m, n), 23, 100)
    want = 3 * (A.astype(np.int64) @ B.astype(np.int64)) - 2 * C.astype(np.int64)
    got = orc.gemm_f64(3.0, A, B, -2.0, C)
    assert np.array_equal(got, want.astype(np.float64))


def test_all_ones_closed_form(orc):
    for m, n, k in [(3, 4, 1), (10, 10, 1000), (1, 1, 4097)]:
        got = orc.gemm_f64(0.5, np.ones((m, k)), np.ones((k, n)), 2.0, np.full((m, n), 0.25))
        assert np.all(got == 0.5 * k + 0.5)


def test_transpose_identity_bitwise(orc):
    A = synth.uniform_pm1((23, 41), 31)
    B = synth.uniform_pm1((41, 17), 32)
    AB = orc.gemm_f64(1.0, A, B)
    BtAt = orc.gemm_f64(1.0, np.ascontiguousarray(B.T), np.ascontiguousarray(A.T))
    assert np.array_equal(AB.T, BtAt)


def test_gamma_bound_medium(orc):
    m, n, k = 40, 30, 2000
    A = synth.uniform_pm1((m, k), 41)
    B = synth.uniform_pm1((k, n), 42)
    C = synth.uniform_pm1((m, n), 43)
    got = orc.gemm_f64(1.5, A, B, 0.5, C)
    ref = orc.gemm_dot2(1.5, A, B, 0.5, C)
    bound = gamma(k + 2) * (1.5 * (np.abs(A) @ np.abs(B)) + 0.5 * np.abs(C))
    assert np.all(np.abs(got - ref) <= bound)
    # and the plain result is not accidentally the double-double one
    assert not np.array_equal(got, ref)


def test_beta_zero_does_not_read_C_and_alpha_zero_does_not_read_AB(orc):
    A = synth.uniform_pm1((6, 5), 1)
    B = synth.uniform_pm1((5, 4), 2)
    Cnan = np.full((6, 4), np.nan)
    got = orc.gemm_f64(2.0, A, B, 0.0, Cnan)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, orc.gemm_f64(2.0, A, B))
    An = np.full((6, 5), np.nan)
    Bn = np.full((5, 4), np.inf)
    C = synth.uniform_pm1((6, 4), 3)
    assert np.array_equal(orc.gemm_f64(0.0, An, Bn, 0.5, C), 0.5 * C)
    assert np.array_equal(orc.gemm_f64(0.0, An, Bn, 0.0, Cnan), np.zeros((6, 4)))
    # k == 0: C = beta*C
    assert np.array_equal(orc.gemm_f64(1.0, np.zeros((6, 0)), np.zeros((0, 4)), 0.5, C), 0.5 * C)


def test_padding_untouched_and_leading_dims(orc):
    m, n, k = 9, 7, 11
    lda, ldb, ldc = 13, 8, 10
    Abuf = np.full((m, lda), np.nan)
    Bbuf = np.full((k, ldb), np.nan)
    Cbuf = np.full((m, ldc), -777.0)
    A = synth.uniform_pm1((m, k), 5)
    B = synth.uniform_pm1((k, n), 6)
    C = synth.uniform_pm1((m, n), 7)
    Abuf[:, :k] = A
    Bbuf[:, :n] = B
    Cbuf[:, :n] = C
    L = orc.lib()
    L.orc_gemm_f64(m, n, k, 1.5, Abuf.ctypes.data, lda, Bbuf.ctypes.data, ldb, 0.5,
                   Cbuf.ctypes.data, ldc, 1)
    assert np.all(Cbuf[:, n:] == -777.0)
    assert np.array_equal(Cbuf[:, :n], orc.gemm_f64(1.5, A, B, 0.5, C))


def test_thread_count_invariance(orc):
    A = synth.uniform_pm1((64, 200), 51)
    B = synth.uniform_pm1((200, 48), 52)
    C = synth.uniform_pm1((64, 48), 53)
    r1 = orc.gemm_f64(1.5, A, B, 0.5, C, nthreads=1)
    r4 = orc.gemm_f64(1.5, A, B, 0.5, C, nthreads=4)
    assert np.array_equal(r1, r4)
    d1 = orc.gemm_dot2(1.5, A, B, 0.5, C, nthreads=1)
    d4 = orc.gemm_dot2(1.5, A, B, 0.5, C, nthreads=4)
    assert np.array_equal(d1, d4)


def test_empty_shapes(orc):
    for m, n, k in itertools.product([0, 1, 3], [0, 2], [0, 4]):
        A = synth.uniform_pm1((m, k), 1)
        B = synth.uniform_pm1((k, n), 2)
        C = synth.uniform_pm1((m, n), 3)
        got = orc.gemm_f64(1.25, A, B, 0.5, C)
        assert got.shape == (m, n)
        if m and n:
            want = 0.5 * C if k == 0 else python_loop_gemm(1.25, A, B, 0.5, C)
            assert np.array_equal(got, want)
