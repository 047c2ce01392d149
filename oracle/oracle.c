/*
 * Oracle for the tiled GEMM C = alpha*A*B + beta*C -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU code that the tests, the smoke check and the
 * benchmark's CPU-baseline leg use to check the GPU library.  It shares no code,
 * header, table or helper with the GPU path, and the product never calls it.
 *
 * Built with  gcc -O2 -mavx2 -mfma -ffp-contract=off -fopenmp  : no product a*b+c
 * is ever fused, so every floating-point step below is one IEEE-754 binary64
 * operation rounded to nearest-even, exactly as written.  fma() is called only
 * where written explicitly (the error-free product of the double-double mode).
 *
 * Layout: every matrix is row-major with a leading dimension in elements
 * (A is m x k, B is k x n, C is m x n).  Sizes are int64_t.
 *
 * Contents
 *   orc_gemm_f64    -- the definition of the operation (paper, Sec. 2, Eq. 1), with
 *                      each C element summed over increasing k; the loop runs in
 *                      i-k-j order, the order of the paper's innermost loop
 *                      (Sec. 5, Listing 2: one row of C updated by a scalar of A times
 *                      a row of B), which gives bit-for-bit the same sums.
 *   orc_gemm_dot2   -- the same result computed with a double-double accumulator
 *                      (Ogita, Rump, Oishi, "Accurate sum and dot product", SIAM J.
 *                      Sci. Comput. 26(6), 2005, algorithm Dot2): a reference whose
 *                      own error is about u^2, used to check paths whose error is
 *                      near the FP64 oracle's own.
 *   orc_split_*     -- the split-precision (Ozaki-style) emulation of an FP64 GEMM:
 *                      exact power-of-two scaling per row of A and column of B, exact
 *                      slicing into small integers, exact integer slice-pair
 *                      products, one rounding to FP64 (Ozaki, Ogita, Oishi, Rump,
 *                      "Error-free transformations of matrix multiplication ...",
 *                      Numer. Algorithms 59, 2012).
 *   orc_crt_gemm    -- the modular-integer emulation (Ozaki scheme II) written as
 *                      its plain definition: operands truncated per row / column,
 *                      their exact product summed in 128-bit integers, one rounding.
 * The FP64 model of the MLP cost model is not here: it is oracle/mlp.py (numpy).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_ERR_NONFINITE 3

/* ------------------------------------------------------------------------- */
/* Plain FP64 GEMM (Eq. 1)                                                    */
/* ------------------------------------------------------------------------- */

/* C = alpha*A*B + beta*C.  BLAS conventions: m==0 or n==0 does nothing; alpha==0
 * or k==0 sets C = beta*C without reading A or B; beta==0 sets C without reading
 * it (a NaN already in C does not propagate).  Padding columns ldc>n are never
 * touched.  nthreads>1 splits the rows over OpenMP threads; the per-element
 * arithmetic is identical for any thread count. */
void orc_gemm_f64(int64_t m, int64_t n, int64_t k, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb,
                  double beta, double *C, int64_t ldc, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads < 1) nthreads = 1;
    if (alpha == 0.0 || k <= 0) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                C[i * ldc + j] = (beta == 0.0) ? 0.0 : beta * C[i * ldc + j];
        return;
    }
#pragma omp parallel num_threads(nthreads)
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t j = 0; j < n; ++j) acc[j] = 0.0;
            for (int64_t p = 0; p < k; ++p) {
                const double a = A[i * lda + p];
                const double *brow = B + p * ldb;
                for (int64_t j = 0; j < n; ++j) acc[j] = acc[j] + a * brow[j];
            }
            double *crow = C + i * ldc;
            if (beta == 0.0) {
                for (int64_t j = 0; j < n; ++j) crow[j] = alpha * acc[j];
            } else {
                for (int64_t j = 0; j < n; ++j) crow[j] = alpha * acc[j] + beta * crow[j];
            }
        }
        free(acc);
    }
}

/* ------------------------------------------------------------------------- */
/* Double-double GEMM (Dot2)                                                  */
/* ------------------------------------------------------------------------- */

/* Knuth's TwoSum: s + e == a + b exactly. */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* Error-free product via one fused multiply-add: p + e == a * b exactly. */
static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* C = alpha*A*B + beta*C with every dot product accumulated as an unevaluated
 * pair (Dot2) and the epilogue also carried in double-double, so that the single
 * final rounding dominates.  Same quick returns as orc_gemm_f64. */
void orc_gemm_dot2(int64_t m, int64_t n, int64_t k, double alpha,
                   const double *A, int64_t lda, const double *B, int64_t ldb,
                   double beta, double *C, int64_t ldc, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads < 1) nthreads = 1;
    if (alpha == 0.0 || k <= 0) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                C[i * ldc + j] = (beta == 0.0) ? 0.0 : beta * C[i * ldc + j];
        return;
    }
#pragma omp parallel num_threads(nthreads)
    {
        double *ph = (double *)malloc(sizeof(double) * (size_t)n);
        double *pl = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t j = 0; j < n; ++j) { ph[j] = 0.0; pl[j] = 0.0; }
            for (int64_t p = 0; p < k; ++p) {
                const double a = A[i * lda + p];
                const double *brow = B + p * ldb;
                for (int64_t j = 0; j < n; ++j) {
                    double h, r, s, q;
                    two_prod(a, brow[j], &h, &r);
                    two_sum(ph[j], h, &s, &q);
                    ph[j] = s;
                    pl[j] = pl[j] + (q + r);
                }
            }
            double *crow = C + i * ldc;
            for (int64_t j = 0; j < n; ++j) {
                /* (ph + pl) * alpha as a pair */
                double h, e;
                two_prod(ph[j], alpha, &h, &e);
                e = e + pl[j] * alpha;
                if (beta == 0.0) {
                    crow[j] = h + e;
                } else {
                    double h2, e2, s, t;
                    two_prod(beta, crow[j], &h2, &e2);
                    two_sum(h, h2, &s, &t);
                    crow[j] = s + (t + (e + e2));
                }
            }
        }
        free(ph);
        free(pl);
    }
}

/* ------------------------------------------------------------------------- */
/* Split-precision emulation of FP64 GEMM (Ozaki scheme)                      */
/* ------------------------------------------------------------------------- */
/*
 * Slice formats (fmt):
 *   0  bfloat16 pieces: every integer |q| <= 2^8 is exact.  First piece b1 = 8
 *      bits, later pieces b = 9 bits, rounding to nearest (the remainder left by
 *      round-to-nearest is at most one half, so one more bit fits under 2^8).
 *   1  FP8 e4m3 pieces: integers |q| <= 2^4 exact; b1 = 4, b = 5, nearest.
 *   2  int8 pieces: integers |q| <= 127; b1 = b = 7 bits, rounding toward zero
 *      (|x| < 2^7 keeps |trunc(x)| <= 127 and leaves a remainder in (-1, 1)).
 *
 * Step 1 (scale, exact): e_i is the exponent with 2^(e_i-1) <= max_p |A_ip| < 2^e_i
 *   (0 for an all-zero row); f_j likewise over column j of B.
 * Step 2 (slice, exact): x = A_ip * 2^(b1 - e_i); q_1 = round(x); r = x - q_1;
 *   for s >= 2: x = r * 2^b; q_s = round(x); r = x - q_s.
 *   Then A_ip = 2^e_i * ( sum_s q_s 2^-(b1 + b(s-1)) + r_S 2^-(b1 + b(S-1)) ).
 * Step 3 (products, exact): G^(s,t) = Q_A^(s) Q_B^(t) in integer arithmetic, for the
 *   pairs with s + t <= S + 1.
 * Step 4 (recombine): level L = s + t has unit 2^-(2 b1 + b (L-2)).  The kept
 *   levels are summed exactly (an integer in units of the smallest level) and
 *   rounded once to FP64, scaled by 2^(e_i + f_j), and the epilogue
 *   alpha*acc + beta*C is applied as in orc_gemm_f64.
 */

int orc_split_bits(int fmt, int *b1, int *b)
{
    if (fmt == 0) { *b1 = 8; *b = 9; return 0; }
    if (fmt == 1) { *b1 = 4; *b = 5; return 0; }
    if (fmt == 2) { *b1 = 7; *b = 7; return 0; }
    return -1;
}

/* 1: slices round to nearest (ties to even); 0: slices round toward zero. */
static int split_nearest(int fmt) { return fmt != 2; }

/* Exponent per row of an r x c row-major matrix (stride ld along rows). */
void orc_split_row_exponents(int64_t r, int64_t c, const double *X, int64_t ld, int32_t *e)
{
    for (int64_t i = 0; i < r; ++i) {
        double mu = 0.0;
        for (int64_t p = 0; p < c; ++p) {
            double v = fabs(X[i * ld + p]);
            if (v > mu) mu = v;
        }
        int ex = 0;
        if (mu > 0.0) (void)frexp(mu, &ex);
        e[i] = ex;
    }
}

/* Exponent per column of an r x c row-major matrix. */
void orc_split_col_exponents(int64_t r, int64_t c, const double *X, int64_t ld, int32_t *f)
{
    for (int64_t j = 0; j < c; ++j) {
        double nu = 0.0;
        for (int64_t p = 0; p < r; ++p) {
            double v = fabs(X[p * ld + j]);
            if (v > nu) nu = v;
        }
        int ex = 0;
        if (nu > 0.0) (void)frexp(nu, &ex);
        f[j] = ex;
    }
}

/* Slices of one value v with exponent ex: writes S integers to q[0..S-1] with
 * stride qs; returns the final remainder (in units of the last piece). */
static double slice_one(double v, int ex, int b1, int b, int nearest, int S, int16_t *q,
                        int64_t qs)
{
    double x = ldexp(v, b1 - ex);
    double r = 0.0;
    for (int s = 0; s < S; ++s) {
        if (s > 0) x = ldexp(r, b);
        double qi = nearest ? nearbyint(x) : trunc(x);
        r = x - qi;
        q[(int64_t)s * qs] = (int16_t)qi;
    }
    return r;
}

/* Slices of A along its rows: Q is S x r x c (slice-major, then row-major). */
void orc_split_slices_rows(int64_t r, int64_t c, const double *X, int64_t ld,
                           const int32_t *e, int fmt, int S, int16_t *Q, double *rem)
{
    int b1, b;
    orc_split_bits(fmt, &b1, &b);
    const int nearest = split_nearest(fmt);
    const int64_t plane = r * c;
    for (int64_t i = 0; i < r; ++i)
        for (int64_t p = 0; p < c; ++p) {
            double rr = slice_one(X[i * ld + p], e[i], b1, b, nearest, S, Q + i * c + p, plane);
            if (rem) rem[i * c + p] = rr;
        }
}

/* Slices of B along its columns: Q is S x r x c (slice-major, then row-major). */
void orc_split_slices_cols(int64_t r, int64_t c, const double *X, int64_t ld,
                           const int32_t *f, int fmt, int S, int16_t *Q, double *rem)
{
    int b1, b;
    orc_split_bits(fmt, &b1, &b);
    const int nearest = split_nearest(fmt);
    const int64_t plane = r * c;
    for (int64_t p = 0; p < r; ++p)
        for (int64_t j = 0; j < c; ++j) {
            double rr = slice_one(X[p * ld + j], f[j], b1, b, nearest, S, Q + p * c + j, plane);
            if (rem) rem[p * c + j] = rr;
        }
}

/* Exact integer product of slice s of A (m x k) and slice t of B (k x n). */
void orc_split_pair_product(int64_t m, int64_t n, int64_t k, const int16_t *QA,
                            const int16_t *QB, int64_t *G)
{
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t acc = 0;
            for (int64_t p = 0; p < k; ++p)
                acc += (int64_t)QA[i * k + p] * (int64_t)QB[p * n + j];
            G[i * n + j] = acc;
        }
}

static int all_finite(int64_t r, int64_t c, const double *X, int64_t ld)
{
    for (int64_t i = 0; i < r; ++i)
        for (int64_t p = 0; p < c; ++p)
            if (!isfinite(X[i * ld + p])) return 0;
    return 1;
}

/* Full split-precision GEMM.  Returns 0, ORC_ERR_NONFINITE (C untouched) when A or
 * B holds a NaN or an infinity, -13 for a bad format, -14 when the exact level
 * sum would not fit the 128-bit accumulator (k too large).  S is the number of
 * pieces per operand. */
int orc_split_gemm(int64_t m, int64_t n, int64_t k, double alpha,
                   const double *A, int64_t lda, const double *B, int64_t ldb,
                   double beta, double *C, int64_t ldc, int fmt, int S, int nthreads)
{
    if (m <= 0 || n <= 0) return ORC_OK;
    if (nthreads < 1) nthreads = 1;
    if (alpha == 0.0 || k <= 0) {
        orc_gemm_f64(m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc, 1);
        return ORC_OK;
    }
    if (!all_finite(m, k, A, lda) || !all_finite(k, n, B, ldb)) return ORC_ERR_NONFINITE;
    int b1, b;
    if (orc_split_bits(fmt, &b1, &b) != 0 || S < 1 || S > 16) return -13;
    /* largest level sum in units of the smallest kept level:
     * (pairs) * D^2 * k * 2^(b (S-1)) must stay below 2^125 */
    {
        double bits = 2.0 * b1 + log2((double)k) + log2((double)S) + (double)b * (S - 1);
        if (bits > 125.0) return -14;
    }

    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *f = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int16_t *QA = (int16_t *)malloc(sizeof(int16_t) * (size_t)(S * m * k));
    int16_t *QB = (int16_t *)malloc(sizeof(int16_t) * (size_t)(S * k * n));
    orc_split_row_exponents(m, k, A, lda, e);
    orc_split_col_exponents(k, n, B, ldb, f);
    orc_split_slices_rows(m, k, A, lda, e, fmt, S, QA, NULL);
    orc_split_slices_cols(k, n, B, ldb, f, fmt, S, QB, NULL);

    /* B slices transposed to n x k per slice so that each level sum runs along
     * contiguous memory; the arithmetic is plain integer and order-free. */
    int16_t *QBt = (int16_t *)malloc(sizeof(int16_t) * (size_t)(S * k * n));
    for (int t = 0; t < S; ++t)
        for (int64_t p = 0; p < k; ++p)
            for (int64_t j = 0; j < n; ++j)
                QBt[(int64_t)t * n * k + j * k + p] = QB[(int64_t)t * k * n + p * n + j];

    const int lowest = 2 * b1 + b * (S - 1);   /* exponent of the unit of level S+1 */
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            __int128 total = 0;
            for (int L = 2; L <= S + 1; ++L) {
                int64_t level = 0;
                for (int s = 1; s <= S; ++s) {
                    int t = L - s;
                    if (t < 1 || t > S) continue;
                    const int16_t *qa = QA + (int64_t)(s - 1) * m * k + i * k;
                    const int16_t *qb = QBt + (int64_t)(t - 1) * n * k + j * k;
                    int64_t g = 0;
                    for (int64_t p = 0; p < k; ++p) g += (int64_t)qa[p] * (int64_t)qb[p];
                    level += g;
                }
                /* level L in units of level S+1 */
                total += (__int128)level * ((__int128)1 << (b * (S + 1 - L)));
            }
            /* one rounding (IEEE conversion of the exact integer), then exact
             * power-of-two scalings */
            double acc = ldexp((double)total, -lowest + e[i] + f[j]);
            double *c = C + i * ldc + j;
            *c = (beta == 0.0) ? alpha * acc : alpha * acc + beta * *c;
        }
    }
    free(QBt);
    free(QB);
    free(QA);
    free(f);
    free(e);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Modular-integer emulation (Ozaki scheme II: Ozaki, Uchino, Imamura 2025).
 *
 * The scheme scales each row of A and each column of B by a power of two,
 * truncates them to integers of at most `bits` bits, and obtains the exact
 * integer product from its residues modulo several small pairwise coprime
 * moduli (Chinese remainder theorem).  The moduli only carry the product; what
 * the scheme computes is fixed by the truncated operands, and that is what this
 * function writes out directly:
 *   e_i, f_j  exponents of the row / column maxima (as orc_split_row_exponents),
 *   A'_ip = trunc(A_ip 2^(bits - e_i)),  B'_pj = trunc(B_pj 2^(bits - f_j)),
 *   C_ij  = round(sum_p A'_ip B'_pj) 2^(e_i + f_j - 2 bits)   (one rounding),
 * then alpha*acc + beta*C as in orc_gemm_f64.  |A'|, |B'| < 2^bits, so the exact
 * sum is below k 2^(2 bits); it is accumulated in 128-bit integers, so the call
 * is refused (-14) when k 2^(2 bits) > 2^125.  Returns ORC_ERR_NONFINITE (C
 * untouched) on NaN / Inf in A or B, -13 for bits outside [1, 62].
 * --------------------------------------------------------------------------- */
int orc_crt_gemm(int64_t m, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc, int bits, int nthreads)
{
    if (m <= 0 || n <= 0) return ORC_OK;
    if (nthreads < 1) nthreads = 1;
    if (alpha == 0.0 || k <= 0) {
        orc_gemm_f64(m, n, 0, alpha, A, lda, B, ldb, beta, C, ldc, 1);
        return ORC_OK;
    }
    if (!all_finite(m, k, A, lda) || !all_finite(k, n, B, ldb)) return ORC_ERR_NONFINITE;
    if (bits < 1 || bits > 62) return -13;
    if (log2((double)k) + 2.0 * bits > 125.0) return -14;

    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *f = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *TA = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * k));
    int64_t *TB = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * k));   /* n x k */
    orc_split_row_exponents(m, k, A, lda, e);
    orc_split_col_exponents(k, n, B, ldb, f);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = 0; p < k; ++p)
            TA[i * k + p] = (int64_t)trunc(ldexp(A[i * lda + p], bits - e[i]));
    for (int64_t p = 0; p < k; ++p)
        for (int64_t j = 0; j < n; ++j)
            TB[j * k + p] = (int64_t)trunc(ldexp(B[p * ldb + j], bits - f[j]));

#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            __int128 total = 0;
            for (int64_t p = 0; p < k; ++p)
                total += (__int128)TA[i * k + p] * (__int128)TB[j * k + p];
            double acc = ldexp((double)total, e[i] + f[j] - 2 * bits);
            double *c = C + i * ldc + j;
            *c = (beta == 0.0) ? alpha * acc : alpha * acc + beta * *c;
        }
    }
    free(TB);
    free(TA);
    free(f);
    free(e);
    return ORC_OK;
}

int orc_num_procs(void) { return omp_get_num_procs(); }
