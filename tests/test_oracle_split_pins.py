"""Pins of the oracle's split-precision (Ozaki) emulation.

What fixes each step, independent of the oracle's own code:
* scale: the exponent inequality 2^(e-1) <= max|x| < 2^e, checked with exact powers;
* slice: the exact reconstruction identity in rational arithmetic and the bound
  |q| <= D of the slice format (a wrong bit count, sign or scale breaks one of them);
* pair products: numpy's int64 matrix product (an independent library routine);
* the full product: a rigorous a-priori error bound against exact rational / Dot2
  references, the monotone gain with more slices, and the 1e-14 normwise target
  on the wide-range stress inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth

U = 2.0 ** -53


def test_slice_format_bits(orc):
    assert orc.split_bits(orc.FMT_BF16) == (8, 9)   # bfloat16: 8 significant bits
    assert orc.split_bits(orc.FMT_E4M3) == (4, 5)   # e4m3: 4 significant bits
    assert orc.split_bits(orc.FMT_INT8) == (7, 7)   # int8: |q| <= 127, truncated


@pytest.mark.parametrize("gen", ["uniform", "wide"])
def test_exponents_bracket_the_row_and_column_maxima(orc, gen):
    f = synth.uniform_pm1 if gen == "uniform" else synth.wide_range
    X = f((37, 53), 5)
    X[3, :] = 0.0
    X[:, 7] = 0.0
    e = orc.split_row_exponents(X)
    for i in range(X.shape[0]):
        mu = np.max(np.abs(X[i]))
        if mu == 0:
            assert e[i] == 0
        else:
            assert np.ldexp(1.0, int(e[i]) - 1) <= mu < np.ldexp(1.0, int(e[i]))
    fcol = orc.split_col_exponents(X)
    for j in range(X.shape[1]):
        nu = np.max(np.abs(X[:, j]))
        if nu == 0:
            assert fcol[j] == 0
        else:
            assert np.ldexp(1.0, int(fcol[j]) - 1) <= nu < np.ldexp(1.0, int(fcol[j]))


@pytest.mark.parametrize("fmt,S", [(0, 6), (0, 3), (1, 11), (1, 5), (2, 8), (2, 3)])
def test_slices_reconstruct_exactly_and_respect_the_bound(orc, fmt, S):
    b1, b = orc.split_bits(fmt)
    D = 2 ** b1 if fmt != 2 else 127
    rmax = 0.5 if fmt != 2 else 1.0
    A = synth.wide_range((9, 13), 77)
    A[2, 5] = 0.0
    A[4, :] = 0.0
    e = orc.split_row_exponents(A)
    Q, rem = orc.split_slices_rows(A, e, fmt, S)
    assert np.all(np.abs(Q.astype(np.int64)) <= D)
    assert np.all(np.abs(rem) <= rmax) and (fmt != 2 or np.all(np.abs(rem) < 1.0))
    for i in range(A.shape[0]):
        for p in range(A.shape[1]):
            acc = Fraction(0)
            for s in range(S):
                acc += Fraction(int(Q[s, i, p])) / Fraction(2) ** (b1 + b * s)
            acc += Fraction(rem[i, p]) / Fraction(2) ** (b1 + b * (S - 1))
            assert Fraction(A[i, p]) == acc * Fraction(2) ** int(e[i])
    # the same for B along its columns
    B = synth.wide_range((13, 7), 78)
    f = orc.split_col_exponents(B)
    QB, remB = orc.split_slices_cols(B, f, fmt, S)
    assert np.all(np.abs(QB.astype(np.int64)) <= D)
    for p in range(B.shape[0]):
        for j in range(B.shape[1]):
            acc = sum((Fraction(int(QB[t, p, j])) / Fraction(2) ** (b1 + b * t) for t in range(S)),
                      Fraction(0))
            acc += Fraction(remB[p, j]) / Fraction(2) ** (b1 + b * (S - 1))
            assert Fraction(B[p, j]) == acc * Fraction(2) ** int(f[j])


def test_slices_are_nearest_integers(orc):
    """rint, not truncation: the first slice of 0.75*2^e with b1 = 8 is 192, and a
    value whose scaled form is x.5 rounds to the even neighbour."""
    A = np.array([[0.75, 0.5 + 2.0 ** -9, 0.5 + 3 * 2.0 ** -9]])
    e = orc.split_row_exponents(A)
    assert e[0] == 0
    Q, _ = orc.split_slices_rows(A, e, 0, 2)
    assert Q[0, 0, 0] == 192
    assert Q[0, 0, 1] == 128          # 128.5 -> 128 (even)
    assert Q[1, 0, 1] == 256          # remainder +0.5 -> 0.5 * 2^9
    assert Q[0, 0, 2] == 130          # 129.5 -> 130 (even)
    assert Q[1, 0, 2] == -256         # remainder -0.5


def test_int8_slices_truncate_toward_zero(orc):
    """b1 = b = 7 with truncation: 0.75 -> 96; 0.5 + 2^-8 -> 64.5 -> 64, remainder
    0.5 -> 64; the negative mirror gives -64, -64 (not -65 / rounding away)."""
    A = np.array([[0.75, 0.5 + 2.0 ** -8, -0.5 - 2.0 ** -8, 0.25 + 2.0 ** -20]])
    e = orc.split_row_exponents(A)
    assert e[0] == 0
    Q, rem = orc.split_slices_rows(A, e, 2, 3)
    assert list(Q[:, 0, 0]) == [96, 0, 0]
    assert list(Q[:, 0, 1]) == [64, 64, 0]
    assert list(Q[:, 0, 2]) == [-64, -64, 0]
    # 0.25 + 2^-20: 32 + 2^-13 -> 32, then 2^-13 * 2^7 = 2^-6 -> 0, then 2^-6*2^7 = 2 -> 2
    assert list(Q[:, 0, 3]) == [32, 0, 2]
    assert np.all(rem[0] == 0.0)


def test_pair_product_equals_numpy_int64(orc):
    QA = synth.integer_valued((23, 300), 1, 256).astype(np.int16)
    QB = synth.integer_valued((300, 19), 2, 256).astype(np.int16)
    G = orc.split_pair_product(QA, QB)
    assert np.array_equal(G, QA.astype(np.int64) @ QB.astype(np.int64))


def split_bound(orc, A, B, fmt, S):
    """A-priori bound on |split(A,B) - A B| per element (alpha=1, beta=0):
    truncation of each operand after S slices (half a unit of the last slice,
    relative to 2^e / 2^f), the dropped pairs s+t > S+1 (each piece below
    2^-b(s-1) relative), and (S+2) FP64 roundings of the recombination."""
    b1, b = orc.split_bits(fmt)
    m, k = A.shape
    n = B.shape[1]
    e = orc.split_row_exponents(A).astype(np.float64)
    f = orc.split_col_exponents(B).astype(np.float64)
    scale = np.exp2(e[:, None] + f[None, :])
    rmax = 0.5 if fmt != 2 else 1.0
    trunc = 2.0 * rmax * 2.0 ** -(b1 + b * (S - 1)) * (1 + 2.0 ** -(b1 + b * (S - 1)))
    dropped = sum(2.0 ** -(b * (s + t - 2)) for s in range(1, S + 1) for t in range(1, S + 1)
                  if s + t > S + 1)
    absAB = np.abs(A) @ np.abs(B)
    return k * scale * (trunc + dropped) + (S + 2) * U * (absAB + k * scale * 2 ** -b1)


@pytest.mark.parametrize("fmt,S", [(0, 6), (0, 4), (1, 11), (1, 7), (2, 8), (2, 5)])
def test_split_within_a_priori_bound_of_exact(orc, fmt, S):
    m, n, k = 5, 4, 9
    A = synth.wide_range((m, k), 91)
    B = synth.wide_range((k, n), 92)
    got = orc.split_gemm(1.0, A, B, fmt=fmt, S=S)
    bound = split_bound(orc, A, B, fmt, S)
    for i in range(m):
        for j in range(n):
            ex = sum((Fraction(A[i, p]) * Fraction(B[p, j]) for p in range(k)), Fraction(0))
            assert abs(Fraction(got[i, j]) - ex) <= Fraction(bound[i, j])


@pytest.mark.parametrize("fmt,S", [(0, 6), (0, 3), (1, 11), (2, 8), (2, 4)])
def test_split_is_the_kept_pairs_exact_sum_rounded_once(orc, fmt, S):
    """Steps 3-4 pinned by exact rational arithmetic: with alpha = 1, beta = 0 the
    result is the exact sum over kept pairs s + t <= S + 1 of the slice products,
    scaled by 2^(e_i + f_j), correctly rounded (Python's float(Fraction) is)."""
    b1, b = orc.split_bits(fmt)
    m, n, k = 4, 3, 11
    A = synth.wide_range((m, k), 71)
    B = synth.wide_range((k, n), 72)
    e = orc.split_row_exponents(A)
    f = orc.split_col_exponents(B)
    QA, _ = orc.split_slices_rows(A, e, fmt, S)
    QB, _ = orc.split_slices_cols(B, f, fmt, S)
    got = orc.split_gemm(1.0, A, B, fmt=fmt, S=S)
    for i in range(m):
        for j in range(n):
            v = Fraction(0)
            for s_ in range(S):
                for t in range(S):
                    if s_ + t + 2 > S + 1:
                        continue
                    g = sum(int(QA[s_, i, p]) * int(QB[t, p, j]) for p in range(k))
                    v += Fraction(g) / Fraction(2) ** (2 * b1 + b * (s_ + t))
            v *= Fraction(2) ** (int(e[i]) + int(f[j]))
            assert got[i, j] == float(v)


def test_split_bound_medium_vs_dot2_and_more_slices_help(orc):
    m, n, k = 32, 24, 700
    A = synth.wide_range((m, k), 93)
    B = synth.wide_range((k, n), 94)
    ref = orc.gemm_dot2(1.0, A, B)
    errs = []
    for S in (2, 3, 4, 5, 6):
        got = orc.split_gemm(1.0, A, B, fmt=0, S=S)
        bound = split_bound(orc, A, B, 0, S)
        assert np.all(np.abs(got - ref) <= bound * (1 + 1e-6) + 4 * U * U * np.abs(A) @ np.abs(B))
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs


def test_split_alpha_beta_epilogue(orc):
    A = synth.uniform_pm1((12, 40), 1)
    B = synth.uniform_pm1((40, 9), 2)
    C = synth.uniform_pm1((12, 9), 3)
    base = orc.split_gemm(1.0, A, B, 0.0, None, fmt=0)
    got = orc.split_gemm(1.5, A, B, 0.5, C, fmt=0)
    assert np.array_equal(got, 1.5 * base + 0.5 * C)
    Cnan = np.full((12, 9), np.nan)
    assert np.array_equal(orc.split_gemm(1.5, A, B, 0.0, Cnan, fmt=0), 1.5 * base)
    assert np.array_equal(orc.split_gemm(0.0, A, B, 0.5, C, fmt=0), 0.5 * C)


def test_split_zero_rows_and_columns(orc):
    A = synth.uniform_pm1((6, 10), 1)
    B = synth.uniform_pm1((10, 5), 2)
    A[2] = 0.0
    B[:, 3] = 0.0
    got = orc.split_gemm(1.0, A, B, fmt=0)
    assert np.all(got[2] == 0.0) and np.all(got[:, 3] == 0.0)
    ref = orc.gemm_dot2(1.0, A, B)
    assert np.linalg.norm(got - ref) <= 1e-15 * np.linalg.norm(ref)


def test_split_nonfinite_raises(orc):
    A = synth.uniform_pm1((4, 4), 1)
    B = synth.uniform_pm1((4, 4), 2)
    A[1, 2] = np.inf
    with pytest.raises(FloatingPointError):
        orc.split_gemm(1.0, A, B)
    A[1, 2] = np.nan
    with pytest.raises(FloatingPointError):
        orc.split_gemm(1.0, A, B)


def test_split_exact_when_one_slice_holds_everything(orc):
    """Integer inputs below 2^7 fit the first bfloat16 slice exactly (q1 = 2a or a
    multiple), so every dropped or truncated term is zero and the result is the
    exact integer product."""
    A = synth.integer_valued((20, 64), 3, 100)
    B = synth.integer_valued((64, 16), 4, 100)
    want = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(orc.split_gemm(1.0, A, B, fmt=0, S=1), want)
    assert np.array_equal(orc.split_gemm(1.0, A, B, fmt=0, S=6), want)


@pytest.mark.slow
def test_split_bf16_meets_1e14_on_wide_range_inputs(orc):
    """The stress distribution of the split-precision workload (entries u*2^e,
    e uniform in [-20, 20]) at a size the oracle finishes in seconds."""
    n = 256
    A = synth.wide_range((n, n), 2001)
    B = synth.wide_range((n, n), 2002)
    ref = orc.gemm_dot2(1.0, A, B, nthreads=8)
    got = orc.split_gemm(1.0, A, B, fmt=0, S=6, nthreads=8)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-14, err
    plain = orc.gemm_f64(1.0, A, B, nthreads=8)
    err_plain = np.linalg.norm(plain - ref) / np.linalg.norm(ref)
    assert err_plain <= 1e-14


def test_fp8_slices_are_nearest_integers(orc):
    """e4m3 slices (b1 = 4, then b = 5 bits) round to nearest, ties to even: the
    first slice of 0.75*2^e is 12; 0.5 + 2^-5 scales to 8.5 -> 8 with remainder +0.5,
    whose second slice is 0.5 * 2^5 = 16; 0.5 + 3*2^-5 scales to 9.5 -> 10 with
    remainder -0.5 -> -16; every slice stays within |q| <= 16."""
    A = np.array([[0.75, 0.5 + 2.0 ** -5, 0.5 + 3 * 2.0 ** -5, -0.5 - 2.0 ** -5]])
    e = orc.split_row_exponents(A)
    assert e[0] == 0
    Q, rem = orc.split_slices_rows(A, e, orc.FMT_E4M3, 3)
    assert list(Q[:, 0, 0]) == [12, 0, 0]
    assert list(Q[:, 0, 1]) == [8, 16, 0]
    assert list(Q[:, 0, 2]) == [10, -16, 0]
    assert list(Q[:, 0, 3]) == [-8, -16, 0]
    assert np.all(rem[0] == 0.0)
    assert np.all(np.abs(Q.astype(np.int64)) <= 16)


@pytest.mark.slow
@pytest.mark.parametrize("fmt,S", [(1, 11), (2, 8)])
def test_split_fp8_and_int8_meet_1e14_on_wide_range_inputs(orc, fmt, S):
    """The FP8 e4m3 and int8 slice models on the stress distribution: within 1e-14
    of the double-double oracle, like the bfloat16 model."""
    n = 256
    A = synth.wide_range((n, n), 2001)
    B = synth.wide_range((n, n), 2002)
    ref = orc.gemm_dot2(1.0, A, B, nthreads=8)
    got = orc.split_gemm(1.0, A, B, fmt=fmt, S=S, nthreads=8)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-14, err
