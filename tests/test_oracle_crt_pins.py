"""Pins of the oracle's modular-integer emulation (Ozaki scheme II).

The scheme's result is fixed by the operands truncated to ``bits`` bits per row /
column and one rounding of their exact product.  What pins each part, independent
of the oracle's own code:
* truncation point: single-element products against a truncation done on the
  integer significand (a different route to the same bits);
* exact product and one rounding: integer-valued inputs against numpy's int64
  product, a hand-built case where one rounding and naive summation differ, and
  brute force in rational arithmetic on tiny inputs;
* scaling and sign: exact invariances (power-of-two scaling, negation, row
  permutation) that a wrong exponent or sign would break;
* accuracy: the a-priori truncation bound against an exact rational product and
  the 1e-14 normwise target on the wide-range inputs;
* the operand width rule k 2^(2 bits) <= 2^123 and the refusals.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth

U = 2.0 ** -53


def _trunc_bits(x: float, bits: int, ex: int) -> float:
    """x truncated toward zero to the multiples of 2^(ex - bits), computed on the
    53-bit integer significand."""
    if x == 0.0:
        return 0.0
    mant, e = math.frexp(abs(x))                 # abs(x) = mant 2^e, mant in [0.5, 1)
    M = int(mant * (1 << 53))                    # exact integer significand
    # abs(x) = M 2^(e - 53); keep multiples of 2^(ex - bits)
    drop = (ex - bits) - (e - 53)
    if drop > 0:
        M = (M >> drop) << drop if drop < 64 else 0
    v = math.ldexp(M, e - 53)
    return -v if x < 0 else v


def test_operand_width_rule(orc):
    for k in [1, 2, 3, 4, 5, 63, 64, 65, 1000, 8192, 8193, 16384, 131072, 10 ** 6]:
        b = orc.crt_bits(k)
        assert k * 2 ** (2 * b) <= 2 ** 123
        assert b == 62 or k * 2 ** (2 * b + 2) > 2 ** 123
    assert orc.crt_bits(8192) == 55


@pytest.mark.parametrize("bits", [1, 2, 7, 20, 33, 52, 53, 55, 60])
def test_truncation_point_single_element(orc, bits):
    xs = list(synth.wide_range((1, 64), 77 + bits)[0]) + [1.0, -1.0, 0.75, 1.0 - 2 ** -53,
                                                         -(1 + 2 ** -40), 2.0 ** -1000]
    for x in xs:
        got = orc.crt_gemm(1.0, np.array([[x]]), np.array([[1.0]]), bits=bits)[0, 0]
        ex = math.frexp(x)[1] if x != 0 else 0
        assert got == _trunc_bits(float(x), bits, ex), (x, bits)


def test_integer_inputs_give_the_exact_product(orc):
    m, n, k = 13, 17, 50
    A = synth.integer_valued((m, k), 3, 1 << 20)
    B = synth.integer_valued((k, n), 4, 1 << 20)
    C = synth.integer_valued((m, n), 5, 1000)
    assert orc.crt_bits(k) >= 21                     # every entry fits: no truncation
    want = 3 * (A.astype(np.int64) @ B.astype(np.int64)) - 2 * C.astype(np.int64)
    assert np.max(np.abs(want)) < 2 ** 53
    got = orc.crt_gemm(3.0, A, B, -2.0, C)
    assert np.array_equal(got, want.astype(np.float64))


def test_one_rounding_of_the_exact_sum(orc):
    # 1 + 2^-53 + 2^-58: one rounding gives 1 + 2^-52; summing in doubles gives 1
    A = np.array([[1.0, 1.0, 1.0]])
    B = np.array([[1.0], [2.0 ** -53], [2.0 ** -58]])
    assert orc.crt_bits(3) == 60                     # 2^-58 is kept at 60 bits
    got = orc.crt_gemm(1.0, A, B)[0, 0]
    assert got == 1.0 + 2.0 ** -52
    assert (1.0 + 2.0 ** -53) + 2.0 ** -58 == 1.0


def test_brute_force_tiny(orc):
    for seed in range(6):
        m, n, k = 3, 4, 5
        A = synth.wide_range((m, k), 300 + seed)
        B = synth.wide_range((k, n), 400 + seed)
        C = synth.uniform_pm1((m, n), 500 + seed)
        bits = [5, 12, 30, 61][seed % 4]
        got = orc.crt_gemm(1.25, A, B, -0.5, C, bits=bits)
        for i in range(m):
            ei = math.frexp(float(np.max(np.abs(A[i]))))[1]
            for j in range(n):
                fj = math.frexp(float(np.max(np.abs(B[:, j]))))[1]
                s = sum(Fraction(_trunc_bits(float(A[i, p]), bits, ei)) *
                        Fraction(_trunc_bits(float(B[p, j]), bits, fj)) for p in range(k))
                acc = float(s)                       # correctly rounded (one rounding)
                want = 1.25 * acc + (-0.5) * float(C[i, j])
                assert got[i, j] == want, (seed, i, j)


def test_exact_invariances(orc):
    m, n, k = 19, 23, 41
    A = synth.wide_range((m, k), 61)
    B = synth.wide_range((k, n), 62)
    base = orc.crt_gemm(1.0, A, B)
    assert np.array_equal(orc.crt_gemm(1.0, -A, B), -base)
    assert np.array_equal(orc.crt_gemm(1.0, A * 2.0 ** 37, B), base * 2.0 ** 37)
    assert np.array_equal(orc.crt_gemm(1.0, A, B * 2.0 ** -29), base * 2.0 ** -29)
    perm = np.arange(m)[::-1]
    assert np.array_equal(orc.crt_gemm(1.0, A[perm], B), base[perm])


def test_truncation_error_bound_against_exact_product(orc):
    m, n, k = 9, 11, 37
    A = synth.wide_range((m, k), 71)
    B = synth.wide_range((k, n), 72)
    for bits in (12, 30, orc.crt_bits(k)):
        got = orc.crt_gemm(1.0, A, B, bits=bits)
        for i in range(m):
            ei = math.frexp(float(np.max(np.abs(A[i]))))[1]
            for j in range(n):
                fj = math.frexp(float(np.max(np.abs(B[:, j]))))[1]
                exact = sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(k))
                bound = (2.0 ** (ei - bits) * np.sum(np.abs(B[:, j])) +
                         2.0 ** (fj - bits) * np.sum(np.abs(A[i])) +
                         k * 2.0 ** (ei + fj - 2 * bits))
                err = abs(Fraction(float(got[i, j])) - exact)
                assert err <= Fraction(bound) * (1 + 4 * U) + Fraction(abs(float(exact))) * U
    # 12 bits is visibly coarser than 30: the width is really applied
    e12 = np.abs(orc.crt_gemm(1.0, A, B, bits=12) - orc.gemm_dot2(1.0, A, B)).max()
    e30 = np.abs(orc.crt_gemm(1.0, A, B, bits=30) - orc.gemm_dot2(1.0, A, B)).max()
    assert e12 > 2.0 ** 10 * e30


def test_wide_range_meets_1e14(orc):
    n = 256
    A = synth.wide_range((n, n), 81)
    B = synth.wide_range((n, n), 82)
    ref = orc.gemm_dot2(1.0, A, B)
    got = orc.crt_gemm(1.0, A, B, nthreads=orc.num_procs())
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-14, err


def test_refusals_and_quick_returns(orc):
    A = synth.uniform_pm1((4, 5), 1)
    B = synth.uniform_pm1((5, 3), 2)
    bad = A.copy()
    bad[1, 2] = np.nan
    with pytest.raises(FloatingPointError):
        orc.crt_gemm(1.0, bad, B)
    with pytest.raises(FloatingPointError):
        orc.crt_gemm(1.0, A, np.where(B > 0, np.inf, B))
    with pytest.raises(ValueError):
        orc.crt_gemm(1.0, A, B, bits=63)
    with pytest.raises(OverflowError):
        orc.crt_gemm(1.0, A, B, bits=62)            # 5 * 2^124 > 2^125
    C = synth.uniform_pm1((4, 3), 3)
    assert np.array_equal(orc.crt_gemm(0.0, A, B, 2.0, C), 2.0 * C)
    Z = np.zeros((4, 5))
    assert np.array_equal(orc.crt_gemm(1.0, Z, B), np.zeros((4, 3)))
