// Split-precision emulation of an FP64 GEMM on low-precision matrix cores
// (Ozaki scheme: Ozaki, Ogita, Oishi, Rump, "Error-free transformations of
// matrix multiplication by using fast routines of matrix multiplication and its
// applications", Numer. Algorithms 59, 2012; on matrix engines: Mukunoki, Ozaki,
// Ogita, Imamura, ISC 2020).
//
// C = alpha*A*B + beta*C with FP64 A, B, C:
//  1. scale    e_i = exponent of max_p |A_ip| (2^(e_i-1) <= max < 2^e_i), f_j the
//              same over column j of B; any NaN/Inf in A or B is reported.
//  2. slice    x = A_ip 2^(b1-e_i); q_1 = round(x); x = (x - q_1) 2^b; q_2 = ...
//              S integer slices per element, exactly representable in the slice
//              format; B is sliced per column and stored transposed, so both
//              operands are k-contiguous.
//  3. products for every pair (s, t) with s + t <= S + 1 the integer product
//              Q_A^(s) Q_B^(t) on matrix cores, summed per level L = s + t.  The
//              sums are exact: bf16 products accumulate in FP32 in chunks small
//              enough that every partial sum is an integer below 2^24 and are then
//              added into two FP64 accumulators that hold exact integers (levels
//              2-4 and 5-7; FP8: 2-6 and 7-12); int8 products accumulate exactly in
//              int32.
//  4. combine  the exact sum of the kept levels is rounded once to FP64,
//              scaled by 2^(e_i + f_j) and the epilogue alpha*v + beta*C applied.
//
// Formats: bf16 slices, b1 = 8, b = 9 bits, round to nearest, S = 6 (21 pairs);
//          FP8 e4m3 slices, b1 = 4, b = 5 bits, round to nearest, S = 11 (66 pairs);
//          int8 slices, b1 = b = 7 bits, round toward zero, S = 8 (36 pairs).
//
// Workspace (device, owned by the library, grown on demand): exponents, a
// non-finite flag and the slices, laid out per row as [row][k-chunk][slice][KC]
// so that one k-chunk of all slices of a row is one contiguous run.
#include <limits.h>

#include <mutex>

#include "mgemm_internal.h"

namespace mgemm {

int32_t set_error(int32_t code, const char *fmt, ...);

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
// 16 bytes as a native vector (HIP's uint4 is a union-based class that the
// compiler cannot keep in registers when held in arrays)
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Slice formats.
// ---------------------------------------------------------------------------
struct FmtBF16 {
    static constexpr int S = 6;         // slices per operand
    static constexpr int B1 = 8;        // bits of the first slice
    static constexpr int B = 9;         // bits of each later slice
    static constexpr bool NEAREST = true;
    static constexpr int KC = 16;       // k per chunk = k of one MFMA step
    static constexpr int ELEM = 2;      // bytes per slice element
    // integer-valued q with |q| <= 256 -> bf16 bits (exact: <= 8 significant bits)
    static __device__ inline uint32_t encode(double q) {
        return __float_as_uint((float)q) >> 16;
    }
};

struct FmtI8 {
    static constexpr int S = 8;
    static constexpr int B1 = 7;
    static constexpr int B = 7;
    static constexpr bool NEAREST = false;
    static constexpr int KC = 32;
    static constexpr int ELEM = 1;
    static __device__ inline uint32_t encode(double q) { return (uint32_t)(uint8_t)(int8_t)(int)q; }
};

struct FmtE4M3 {
    static constexpr int S = 11;
    static constexpr int B1 = 4;
    static constexpr int B = 5;
    static constexpr bool NEAREST = true;
    static constexpr int KC = 64;       // k of one FP8 MFMA step
    static constexpr int ELEM = 1;
    // integer-valued q with |q| <= 16 -> FP8 e4m3 byte (OCP: exponent bias 7, three
    // mantissa bits; exact, at most 4 significant bits)
    static __device__ inline uint32_t encode(double q) {
        if (q == 0.0) return 0u;
        const uint32_t f = __float_as_uint((float)q);
        const uint32_t ex = ((f >> 23) & 0xFFu) - 127u + 7u;
        return ((f >> 24) & 0x80u) | (ex << 3) | ((f >> 20) & 7u);
    }
};

// bytes of one (row, k-chunk) run: all S slices of KC elements
template <typename F> constexpr int run_bytes() { return F::S * F::KC * F::ELEM; }

constexpr int KPAD = 64;     // k padded to a multiple of 64 (slice-B transpose tile)
constexpr int PBM = 64;      // pair kernel tile rows
constexpr int PBN = 128;     // pair kernel tile columns

// ---------------------------------------------------------------------------
// 1. Scale.
// ---------------------------------------------------------------------------
__global__ void split_init_kernel(int *fexp, int64_t np, int *flag) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < np;
         j += (int64_t)gridDim.x * blockDim.x)
        fexp[j] = INT_MIN;
    if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
}

__device__ inline int exponent_of(double mx) {
    int ex = 0;
    if (mx > 0.0) (void)frexp(mx, &ex);
    return ex;
}

// One 256-thread block per row (grid-stride over rows).
__global__ void __launch_bounds__(256)
split_row_scale_kernel(const double *__restrict__ A, int64_t m, int64_t k, int64_t lda,
                       int *__restrict__ e, int *flag) {
    __shared__ double red[4];
    __shared__ int bad_any[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        double mx = 0.0;
        int bad = 0;
        const double *row = A + i * lda;
        for (int64_t p = tid; p < k; p += 256) {
            double v = row[p];
            if (!isfinite(v)) bad = 1;
            else mx = fmax(mx, fabs(v));
        }
        for (int off = 32; off > 0; off >>= 1) {
            mx = fmax(mx, __shfl_xor(mx, off));
            bad |= __shfl_xor(bad, off);
        }
        if (lane == 0) { red[wave] = mx; bad_any[wave] = bad; }
        __syncthreads();
        if (tid == 0) {
            double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            if (bad_any[0] | bad_any[1] | bad_any[2] | bad_any[3]) *flag = 1;
            e[i] = exponent_of(t);
        }
        __syncthreads();
    }
}

// Thread per column, 64 rows per block row; exponents merged with atomicMax
// (the exponent is non-decreasing in |x|).  Untouched (all-zero) columns keep
// INT_MIN and are read as exponent 0.
constexpr int COL_ROWS = 64;

__global__ void __launch_bounds__(256)
split_col_scale_kernel(const double *__restrict__ B, int64_t k, int64_t n, int64_t ldb,
                       int *__restrict__ fexp, int *flag) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const int64_t nyb = (k + COL_ROWS - 1) / COL_ROWS;
    for (int64_t yb = blockIdx.y; yb < nyb; yb += gridDim.y) {
        const int64_t p0 = yb * COL_ROWS;
        const int64_t p1 = p0 + COL_ROWS < k ? p0 + COL_ROWS : k;
        double mx = 0.0;
        int bad = 0;
        for (int64_t p = p0; p < p1; ++p) {
            double v = B[p * ldb + j];
            if (!isfinite(v)) bad = 1;
            else mx = fmax(mx, fabs(v));
        }
        if (bad) *flag = 1;
        if (mx > 0.0) atomicMax(fexp + j, exponent_of(mx));
    }
}

// ---------------------------------------------------------------------------
// 2. Slice.
// ---------------------------------------------------------------------------
template <typename F>
__device__ inline double slice_round(double x) {
    return F::NEAREST ? rint(x) : trunc(x);
}

// 8 consecutive k values of one row of A -> S slices; rows >= m and k >= k are 0.
template <typename F>
__global__ void __launch_bounds__(256)
split_slice_a_kernel(const double *__restrict__ A, int64_t m, int64_t k, int64_t lda,
                     const int *__restrict__ e, uint8_t *__restrict__ QA, int64_t mp, int64_t kp) {
    const int64_t groups_per_row = kp / 8;
    const int64_t total = mp * groups_per_row;
    const int64_t nch = kp / F::KC;
    for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
         gid += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = gid / groups_per_row;
        const int64_t p0 = (gid - i * groups_per_row) * 8;
        const int ex = i < m ? e[i] : 0;
        double x[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t p = p0 + v;
            x[v] = (i < m && p < k) ? ldexp(A[i * lda + p], F::B1 - ex) : 0.0;
        }
        uint8_t *dst = QA + ((i * nch + p0 / F::KC) * F::S) * F::KC * F::ELEM +
                       (p0 % F::KC) * F::ELEM;
#pragma unroll
        for (int s = 0; s < F::S; ++s) {
            uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const double q = slice_round<F>(x[v]);
                x[v] = (x[v] - q) * (double)(1 << F::B);
                const uint32_t c = F::encode(q);
                if (F::ELEM == 2) w[v >> 1] |= c << (16 * (v & 1));
                else w[v >> 2] |= c << (8 * (v & 3));
            }
            uint8_t *d = dst + (int64_t)s * F::KC * F::ELEM;
            if (F::ELEM == 2) *(uint4 *)d = make_uint4(w[0], w[1], w[2], w[3]);
            else *(uint2 *)d = make_uint2(w[0], w[1]);
        }
    }
}

// 64 (k) x 64 (n) tile of B through LDS; thread (j, 16 consecutive k) -> S slices
// of column j stored k-contiguous.
template <typename F>
__global__ void __launch_bounds__(256)
split_slice_b_kernel(const double *__restrict__ B, int64_t k, int64_t n, int64_t ldb,
                     const int *__restrict__ fexp, uint8_t *__restrict__ QB, int64_t kp) {
    __shared__ double tile[64][65];
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int64_t p0 = (int64_t)blockIdx.y * 64;
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int pr = idx >> 6, jc = idx & 63;
        const int64_t p = p0 + pr, j = j0 + jc;
        tile[pr][jc] = (p < k && j < n) ? B[p * ldb + j] : 0.0;
    }
    __syncthreads();
    const int jc = tid >> 2;
    const int pg = (tid & 3) * 16;
    const int64_t j = j0 + jc;
    const int fe = j < n ? fexp[j] : INT_MIN;
    const int ex = fe == INT_MIN ? 0 : fe;
    double x[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) x[v] = ldexp(tile[pg + v][jc], F::B1 - ex);
    const int64_t nch = kp / F::KC;
    const int64_t pabs = p0 + pg;
    uint8_t *dst = QB + ((j * nch + pabs / F::KC) * F::S) * F::KC * F::ELEM +
                   (pabs % F::KC) * F::ELEM;
#pragma unroll
    for (int s = 0; s < F::S; ++s) {
        uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const double q = slice_round<F>(x[v]);
            x[v] = (x[v] - q) * (double)(1 << F::B);
            const uint32_t c = F::encode(q);
            if (F::ELEM == 2) w[v >> 1] |= c << (16 * (v & 1));
            else w[v >> 2] |= c << (8 * (v & 3));
        }
        uint8_t *d = dst + (int64_t)s * F::KC * F::ELEM;
        if (F::ELEM == 2) {
            ((uint4 *)d)[0] = make_uint4(w[0], w[1], w[2], w[3]);
            ((uint4 *)d)[1] = make_uint4(w[4], w[5], w[6], w[7]);
        } else {
            *(uint4 *)d = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

// ---------------------------------------------------------------------------
// 3-4. Slice-pair products and recombination.
// ---------------------------------------------------------------------------
// Work-group: 8 waves (2 x 4) own a 64 x 128 tile of C; each wave one 32 x 32
// block (one 32x32 MFMA accumulator per level).  Per k-chunk the S slices of the
// 64 A rows and 128 B columns are staged in LDS (double buffered); the 16-byte
// units of one row are padded to an odd count so the fragment reads of 16
// consecutive rows hit distinct banks.
struct PairArgs {
    const uint8_t *QA;
    const uint8_t *QB;
    const int *e;
    const int *fexp;
    double *C;
    int64_t m, n, ldc;
    int64_t nch;        // k-chunks per row in the slice layout
    int64_t ch0, ch1;   // chunk range of this pass
    double alpha, beta;
    int tiles_m, tiles_n;
    double *sums;       // FP8 pair kernel: exact level sums, 32 per lane (else unused)
};

// 32x32 MFMA accumulator element r of lane l -> (row, column) in the wave block
__device__ inline int acc_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Stores the combined value of one element: v = fma(hi, 2^-lo_hi_shift ...)
__device__ inline void store_c(const PairArgs &a, int64_t row, int64_t col, double v) {
    if (row >= a.m || col >= a.n) return;
    const int fe = a.fexp[col];
    const int ex = a.e[row] + (fe == INT_MIN ? 0 : fe);
    const double val = ldexp(v, ex);
    double *c = a.C + row * a.ldc + col;
    if (a.beta == 0.0) {
        *c = a.alpha * val;
    } else {
#pragma clang fp contract(off)
        *c = a.alpha * val + a.beta * *c;
    }
}

template <typename F>
struct PairTile {
    static constexpr int UNITS = run_bytes<F>() / 16;   // 16-byte units per row run
    static constexpr int SROW = UNITS + 1;               // padded LDS row (odd)
    static constexpr int NT = 512;
    static constexpr int TOTAL_UNITS = (PBM + PBN) * UNITS;
    static constexpr int LOADS = (TOTAL_UNITS + NT - 1) / NT;
};

template <typename F>
__device__ __attribute__((always_inline)) inline void pair_load(const PairArgs &a, int64_t m0, int64_t n0, int64_t ch,
                                 u32x4 (&stage)[PairTile<F>::LOADS]) {
    typedef PairTile<F> P;
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < P::LOADS; ++it) {
        const int u = tid + it * P::NT;
        if (u < P::TOTAL_UNITS) {
            const u32x4 *src;
            if (u < PBM * P::UNITS) {
                const int row = u / P::UNITS, c = u % P::UNITS;
                src = (const u32x4 *)(a.QA + ((m0 + row) * a.nch + ch) * run_bytes<F>()) + c;
            } else {
                const int v = u - PBM * P::UNITS;
                const int row = v / P::UNITS, c = v % P::UNITS;
                src = (const u32x4 *)(a.QB + ((n0 + row) * a.nch + ch) * run_bytes<F>()) + c;
            }
            stage[it] = *src;
        }
    }
}

template <typename F>
__device__ __attribute__((always_inline)) inline void pair_store(u32x4 *sA, u32x4 *sB, const u32x4 (&stage)[PairTile<F>::LOADS]) {
    typedef PairTile<F> P;
    const int tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < P::LOADS; ++it) {
        const int u = tid + it * P::NT;
        if (u < P::TOTAL_UNITS) {
            if (u < PBM * P::UNITS) {
                const int row = u / P::UNITS, c = u % P::UNITS;
                sA[row * P::SROW + c] = stage[it];
            } else {
                const int v = u - PBM * P::UNITS;
                const int row = v / P::UNITS, c = v % P::UNITS;
                sB[row * P::SROW + c] = stage[it];
            }
        }
    }
}

// bf16: six FP32 level accumulators, flushed exactly into FP64 (hi: levels 2-4 in
// units of level 4; lo: levels 5-7 in units of level 7).  Flush periods (in
// 16-deep chunks) keep every FP32 partial sum an integer of magnitude <= 2^24:
// level L has (L-1) pairs of products <= 2^16, so it may run 256/(L-1) k-steps.
__global__ void __launch_bounds__(512)
split_pairs_bf16_kernel(PairArgs a) {
    typedef FmtBF16 F;
    typedef PairTile<F> P;
    __shared__ u32x4 sA[2][PBM * P::SROW];
    __shared__ u32x4 sB[2][PBN * P::SROW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, a.tiles_m, a.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * PBM, n0 = (int64_t)tn * PBN;

    v16f acc[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) acc[l] = v16f{};
    double hi[16], lo[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) { hi[r] = 0.0; lo[r] = 0.0; }

    const int r32 = lane & 31, kh = lane >> 5;
    const int a_off = (wm * 32 + r32) * P::SROW + kh;
    const int b_off = (wn * 32 + r32) * P::SROW + kh;

    u32x4 stage[P::LOADS];
    pair_load<F>(a, m0, n0, a.ch0, stage);
    pair_store<F>(sA[0], sB[0], stage);
    __syncthreads();

    constexpr int PERIOD[6] = {16, 8, 4, 4, 2, 2};
    for (int64_t ch = a.ch0; ch < a.ch1; ++ch) {
        const int cur = (int)((ch - a.ch0) & 1);
        const bool more = ch + 1 < a.ch1;
        if (more) pair_load<F>(a, m0, n0, ch + 1, stage);

        v8bf fa[6], fb[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            fa[s] = __builtin_bit_cast(v8bf, sA[cur][a_off + 2 * s]);
            fb[s] = __builtin_bit_cast(v8bf, sB[cur][b_off + 2 * s]);
        }
#pragma unroll
        for (int lv = 0; lv < 6; ++lv)
#pragma unroll
            for (int s = 0; s <= lv; ++s)
                acc[lv] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[lv - s], acc[lv], 0, 0, 0);

        const int64_t done = ch - a.ch0 + 1;
#pragma unroll
        for (int lv = 0; lv < 6; ++lv) {
            if (done % PERIOD[lv] == 0 || !more) {
                // hi holds levels 2..4 (lv 0..2) in units of level 4, lo levels
                // 5..7 (lv 3..5) in units of level 7: both stay exact integers
                const double sc = (double)(1 << (9 * (2 - (lv % 3))));
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if (lv < 3) hi[r] = fma((double)acc[lv][r], sc, hi[r]);
                    else lo[r] = fma((double)acc[lv][r], sc, lo[r]);
                }
                acc[lv] = v16f{};
            }
        }
        if (more) pair_store<F>(sA[cur ^ 1], sB[cur ^ 1], stage);
        __syncthreads();
    }

    // exact value = hi 2^-34 + lo 2^-61, rounded once
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const double v = fma(hi[r], 0x1p-34, lo[r] * 0x1p-61);
        store_c(a, m0 + wm * 32 + acc_row(lane, r), n0 + wn * 32 + r32, v);
    }
}

// int8, pipelined: one wave per SIMD (4 waves as 2 x 2), each wave a 64 x 32
// block of C held as two 32x32 accumulators per level (256 accumulator
// registers).  Three LDS stages are filled by direct global->LDS loads (no
// staging registers).  While the products of chunk c run, each fragment register
// is refilled with chunk c+1 right after its last use in chunk c, and chunk c+2
// is loading into the third stage; one barrier per chunk publishes a stage whose
// loads were issued a whole chunk earlier.  Slice buffers are addressed with
// 32-bit offsets (each below 4 GiB, checked on the host).
constexpr int Q_BM = 128, Q_BN = 64;
constexpr int Q_UNITS = 16;                              // units of one row run
constexpr int Q_SROW = 17;                               // padded LDS row (units)
constexpr int Q_STAGE = (Q_BM + Q_BN) * Q_SROW;          // 3264 units per stage
constexpr int Q_LOADS = (Q_STAGE + 255) / 256;           // load instructions per wave

// Load instruction i of chunk ch into stage (the last instruction only for the
// waves whose units lie inside the stage).
__device__ __attribute__((always_inline)) inline void q_issue_one(
    const PairArgs &a, int i, uint32_t a_row0, uint32_t b_row0, uint32_t ch, u32x4 *stage,
    int wave, int lane) {
    const uint32_t run = 256u, stride = (uint32_t)a.nch * 256u;
    const int first = i * 256 + wave * 64;            // first unit of this wave instruction
    if (first >= Q_STAGE) return;                     // uniform per wave
    const int u = first + lane;
    const uint8_t *src;
    if (u < Q_BM * Q_SROW) {
        const int row = u / Q_SROW, c = u % Q_SROW;
        src = a.QA + ((a_row0 + row) * stride + ch * run + (uint32_t)(c < Q_UNITS ? c : Q_UNITS - 1) * 16u);
    } else {
        const int v = u - Q_BM * Q_SROW;
        const int row = v / Q_SROW, c = v % Q_SROW;
        src = a.QB + ((b_row0 + row) * stride + ch * run + (uint32_t)(c < Q_UNITS ? c : Q_UNITS - 1) * 16u);
    }
    __builtin_amdgcn_global_load_lds(
        (const void *)src, (__attribute__((address_space(3))) void *)(stage + first), 16, 0, 0);
}

__device__ __attribute__((always_inline)) inline void q_issue_loads(
    const PairArgs &a, uint32_t a_row0, uint32_t b_row0, uint32_t ch, u32x4 *stage, int wave,
    int lane) {
#pragma unroll
    for (int i = 0; i < Q_LOADS; ++i) q_issue_one(a, i, a_row0, b_row0, ch, stage, wave, lane);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
split_pairs_i8_pipe_kernel(PairArgs a) {
    __shared__ u32x4 lds[3 * Q_STAGE];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, a.tiles_m, a.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * Q_BM, n0 = (int64_t)tn * Q_BN;
    const int r32 = lane & 31, kh = lane >> 5;
    const int a_off0 = (wm * 64 + r32) * Q_SROW + kh;            // m-tile 0
    const int a_off1 = (wm * 64 + 32 + r32) * Q_SROW + kh;       // m-tile 1
    const int b_off = Q_BM * Q_SROW + (wn * 32 + r32) * Q_SROW + kh;

    v16i acc[8][2];
#pragma unroll
    for (int l = 0; l < 8; ++l) {
        acc[l][0] = v16i{};
        acc[l][1] = v16i{};
    }
    v4i fa[8][2], fb[8];

    const uint32_t ar0 = (uint32_t)m0, br0 = (uint32_t)n0;
    // products of the current chunk; every fragment is reloaded from the next
    // stage right after its last use (after the last chunk the reloads read a
    // stale stage and are never used -- they stay inside the LDS allocation),
    // and the loads of chunk lc into stage lst go out one every two slice pairs
    auto products = [&](const u32x4 *nst, uint32_t lc, u32x4 *lst) {
        int slot = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
#pragma unroll
            for (int t = 7 - s; t >= 0; --t) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
                    acc[s + t][mt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[s][mt], fb[t],
                                                                            acc[s + t][mt], 0, 0, 0);
                // fb[t] is last used by slice s = 7 - t; the scheduling barriers
                // keep each reload and load next to the products it overlaps
                if (t == 7 - s) fb[t] = __builtin_bit_cast(v4i, nst[b_off + 2 * t]);
                if (slot % 2 == 0 && slot / 2 < Q_LOADS)
                    q_issue_one(a, slot / 2, ar0, br0, lc, lst, wave, lane);
                ++slot;
                __builtin_amdgcn_sched_barrier(0);
            }
            fa[s][0] = __builtin_bit_cast(v4i, nst[a_off0 + 2 * s]);
            fa[s][1] = __builtin_bit_cast(v4i, nst[a_off1 + 2 * s]);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    const uint32_t c0 = (uint32_t)a.ch0, c1 = (uint32_t)a.ch1;
    q_issue_loads(a, ar0, br0, c0, lds, wave, lane);
    q_issue_loads(a, ar0, br0, c0 + 1 < c1 ? c0 + 1 : c0, lds + Q_STAGE, wave, lane);
    __builtin_amdgcn_s_waitcnt(0x0F70);          // vmcnt(0)
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        fa[s][0] = __builtin_bit_cast(v4i, lds[a_off0 + 2 * s]);
        fa[s][1] = __builtin_bit_cast(v4i, lds[a_off1 + 2 * s]);
        fb[s] = __builtin_bit_cast(v4i, lds[b_off + 2 * s]);
    }
    int st = 0;                                   // stage of chunk c
    for (uint32_t c = c0; c < c1; ++c) {
        // publish chunk c+1 (own loads done, then everyone's)
        __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0)
        __syncthreads();
        const int st1 = st == 2 ? 0 : st + 1;
        const int st2 = st1 == 2 ? 0 : st1 + 1;
        // chunk c+2 (past the end: the last chunk again, in bounds, never used)
        products(lds + st1 * Q_STAGE, c + 2 < c1 ? c + 2 : c1 - 1, lds + st2 * Q_STAGE);
        st = st1;
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);          // vmcnt(0): no load lands after this point

#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double hi = (double)acc[0][mt][r] * 0x1p21;
            hi = hi + (double)acc[1][mt][r] * 0x1p14;
            hi = hi + (double)acc[2][mt][r] * 0x1p7;
            hi = hi + (double)acc[3][mt][r];
            double lo = (double)acc[4][mt][r] * 0x1p21;
            lo = lo + (double)acc[5][mt][r] * 0x1p14;
            lo = lo + (double)acc[6][mt][r] * 0x1p7;
            lo = lo + (double)acc[7][mt][r];
            const double v = fma(hi, 0x1p-35, lo * 0x1p-63);
            store_c(a, m0 + wm * 64 + mt * 32 + acc_row(lane, r), n0 + wn * 32 + r32, v);
        }
}

// bf16, pipelined: 8 waves (2 x 4, two per SIMD) own a 64 x 128 tile of C, each
// wave a 32 x 32 block held as one 32x32 FP32 accumulator per level plus the
// exact FP64 hi / lo sums.  Four LDS stages (one k-chunk of all 6 slices of the
// tile's 64 A rows and 128 B columns each) are filled by direct global->LDS loads
// three chunks ahead, spread over the products; fragments are refilled from the
// next stage right after their last use.  Each level is flushed into hi / lo at
// most every 16, 8, 4, 4, 2, 2 chunks; the pass's chunk range is a multiple of
// 16 (k padded with zero slices).
constexpr int R_BM = 64, R_BN = 128;
constexpr int R_THREADS = 512;
constexpr int R_UNITS = 12;                              // units of one row run (6 x 32 B)
constexpr int R_SROW = 13;                               // padded LDS row (units)
constexpr int R_AUNITS = R_BM * R_SROW;                  // 832 units
constexpr int R_STAGE = (R_BM + R_BN) * R_SROW;          // 2496 units per stage
constexpr int R_LOADS = (R_STAGE + R_THREADS - 1) / R_THREADS;   // 5 load instructions per lane
constexpr int R_NST = 4;
constexpr int R_BLOCK = 16;                              // chunks per flush cycle
static_assert(R_AUNITS % 64 == 0 && R_STAGE % 64 == 0, "a wave's loads lie in one operand");
static_assert(R_NST * R_STAGE * 16 <= 163840, "LDS");

__global__ void __launch_bounds__(R_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
split_pairs_bf16_pipe_kernel(PairArgs a) {
    __shared__ u32x4 lds[R_NST * R_STAGE];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 2, wn = wave & 3;
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, a.tiles_m, a.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * R_BM, n0 = (int64_t)tn * R_BN;
    const int r32 = lane & 31, kh = lane >> 5;
    const int a_off = (wm * 32 + r32) * R_SROW + kh;
    const int b_off = R_AUNITS + (wn * 32 + r32) * R_SROW + kh;

    // per-lane source offsets (bytes, chunk 0) of each load instruction; the
    // slices of one row are nch runs of 192 bytes
    const uint32_t stride = (uint32_t)a.nch * 192u;
    uint32_t off[R_LOADS];
#pragma unroll
    for (int i = 0; i < R_LOADS; ++i) {
        const int u = i * R_THREADS + wave * 64 + lane;
        const int v = u < R_AUNITS ? u : u - R_AUNITS;
        const int row = v / R_SROW, c = v % R_SROW;
        const uint32_t row0 = u < R_AUNITS ? (uint32_t)m0 : (uint32_t)n0;
        off[i] = (row0 + (uint32_t)row) * stride + (uint32_t)(c < R_UNITS ? c : R_UNITS - 1) * 16u;
    }
    // load instruction i of chunk ch into stage st (the last instruction only
    // for the waves whose units lie inside the stage)
    auto issue_one = [&](int i, uint32_t ch, int st) {
        const int first = i * R_THREADS + wave * 64;             // uniform per wave
        if ((i + 1) * R_THREADS > R_STAGE && first >= R_STAGE) return;
        const uint8_t *src = (first < R_AUNITS ? a.QA : a.QB) + (off[i] + ch * 192u);
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (__attribute__((address_space(3))) void *)(lds + st * R_STAGE + first),
                                         16, 0, 0);
    };
    // waves whose last instruction lies inside the stage issue R_LOADS loads per
    // chunk, the others one fewer
    const bool full_loads = (R_LOADS - 1) * R_THREADS + wave * 64 < R_STAGE;

    v16f acc[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) acc[l] = v16f{};
    double hi[16], lo[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) hi[r] = lo[r] = 0.0;
    v8bf fa[6], fb[6];

    // products of one chunk (21 slice pairs); fragments are refilled from the
    // next stage after their last use, and the loads of chunk lc into stage ls go
    // out one every four slice pairs
    auto products = [&](const u32x4 *nst, uint32_t lc, int ls) {
        int slot = 0;
#pragma unroll
        for (int s = 0; s < 6; ++s) {
#pragma unroll
            for (int t = 5 - s; t >= 0; --t) {
                acc[s + t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[s], fb[t], acc[s + t], 0, 0, 0);
                if (t == 5 - s) fb[t] = __builtin_bit_cast(v8bf, nst[b_off + 2 * t]);
                if (slot % 4 == 0 && slot / 4 < R_LOADS) issue_one(slot / 4, lc, ls);
                ++slot;
                __builtin_amdgcn_sched_barrier(0);
            }
            fa[s] = __builtin_bit_cast(v8bf, nst[a_off + 2 * s]);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // hi holds levels 2..4 (lv 0..2) in units of level 4, lo levels 5..7 (lv 3..5)
    // in units of level 7: both stay exact integers
    auto flush = [&](int lv) {
        const double sc = (double)(1 << (9 * (2 - (lv % 3))));
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (lv < 3) hi[r] = fma((double)acc[lv][r], sc, hi[r]);
            else lo[r] = fma((double)acc[lv][r], sc, lo[r]);
        }
        acc[lv] = v16f{};
    };

    const uint32_t c0 = (uint32_t)a.ch0;
    const int nch = (int)(a.ch1 - a.ch0);         // a multiple of R_BLOCK
    const uint32_t clast = c0 + (uint32_t)nch - 1;
#pragma unroll
    for (int c = 0; c < R_NST - 1; ++c) {
        const uint32_t ch = c0 + (uint32_t)c <= clast ? c0 + (uint32_t)c : clast;
#pragma unroll
        for (int i = 0; i < R_LOADS; ++i) issue_one(i, ch, c);
    }
    // chunk 0 landed; two chunks' loads may remain
    if (full_loads) __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * R_LOADS));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * (R_LOADS - 1)));
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        fa[s] = __builtin_bit_cast(v8bf, lds[a_off + 2 * s]);
        fb[s] = __builtin_bit_cast(v8bf, lds[b_off + 2 * s]);
    }
    // Level lv is flushed before chunk c when (c + wm) is a multiple of PERIOD[lv]
    // and once more after the last chunk, so it never sums more than PERIOD[lv]
    // chunks.  The one-chunk offset between the two waves of a SIMD (wm = 0, 1)
    // and the flush at the start of a chunk let one wave's flush run on the
    // vector unit while the other wave's products keep the matrix core busy.
    constexpr int PERIOD[6] = {16, 8, 4, 4, 2, 2};
    for (int b = 0; b < nch; b += R_BLOCK) {
#pragma unroll 1
        for (int u = 0; u < R_BLOCK; ++u) {
            // chunk c = b + u (stage u % 4): chunk c+1 landed, one chunk may remain
            if (full_loads) __builtin_amdgcn_s_waitcnt(vmcnt_imm(R_LOADS));
            else __builtin_amdgcn_s_waitcnt(vmcnt_imm(R_LOADS - 1));
            __syncthreads();
            const int ph = u + wm;                // b is a multiple of every period
#pragma unroll
            for (int lv = 0; lv < 6; ++lv)
                if ((ph & (PERIOD[lv] - 1)) == 0) flush(lv);
            const uint32_t next = c0 + (uint32_t)(b + u + 3);
            // chunk c+3 into the stage of chunk c-1 (past the end: the last
            // chunk again, in bounds and never used)
            products(lds + ((u + 1) & 3) * R_STAGE, next <= clast ? next : clast, (u + 3) & 3);
        }
    }
#pragma unroll
    for (int lv = 0; lv < 6; ++lv) flush(lv);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));     // no load lands after this point

    // exact value = hi 2^-34 + lo 2^-61, rounded once
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const double v = fma(hi[r], 0x1p-34, lo[r] * 0x1p-61);
        store_c(a, m0 + wm * 32 + acc_row(lane, r), n0 + wn * 32 + r32, v);
    }
}

// FP8 e4m3: 4 waves (2 x 2, one per SIMD) own a 64 x 64 tile of C, each wave a
// 32 x 32 block held as one 32x32 FP32 accumulator per level (11 levels).  A
// k-chunk (64 k) of all 11 slices of the tile's 64 A rows sits in one of two A
// stages, of its 64 B columns in the one B stage.  At the start of a chunk every
// wave copies its 11 B fragments into registers; once all have, the next chunk's
// direct loads fill the B stage and the other A stage while the 66 products run,
// the A fragments being read row by row from the current A stage.  Products are
// at most 16 x 16 = 2^8, so each level's FP32 sum stays an exact integer below
// 2^24 for 64 chunks (11 x 64 x 64 x 2^8 < 2^24); it is then added into the exact
// FP64 sums hi (levels 2-6 in units of level 6) and lo (levels 7-12 in units of
// level 12).  Slice buffers are addressed with 32-bit offsets (each below 4 GiB,
// checked on the host).
constexpr int E_BM = 64, E_BN = 64;
constexpr int E_THREADS = 256;
constexpr int E_UNITS = 44;                              // units of one row run (11 x 64 B)
constexpr int E_SROW = 45;                               // padded LDS row (units)
constexpr int E_AUNITS = E_BM * E_SROW;                  // 2880 units per A stage
constexpr int E_BUNITS = E_BN * E_SROW;                  // 2880 units in the B stage
constexpr int E_UNITS_CHUNK = E_AUNITS + E_BUNITS;       // units loaded per chunk
constexpr int E_LOADS = (E_UNITS_CHUNK + E_THREADS - 1) / E_THREADS;   // 23 per lane
constexpr int E_FLUSH = 64;                              // chunks between flushes
static_assert(E_AUNITS % 64 == 0 && E_UNITS_CHUNK % 64 == 0, "a wave's loads lie in one operand");
static_assert(11 * E_FLUSH * 64 * 256 < (1 << 24), "FP32 level sums stay exact");
static_assert((2 * E_AUNITS + E_BUNITS) * 16 <= 163840, "LDS");

typedef int v8i_t __attribute__((ext_vector_type(8)));

__global__ void __launch_bounds__(E_THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
split_pairs_e4m3_kernel(PairArgs a) {
    __shared__ u32x4 lds[2 * E_AUNITS + E_BUNITS];      // A stage 0, A stage 1, B stage

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, a.tiles_m, a.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * E_BM, n0 = (int64_t)tn * E_BN;
    const int r32 = lane & 31, kh = lane >> 5;
    // fragment of slice s: 32 bytes (units 4s + 2kh, +1) of the wave's row / column
    const int a_off = (wm * 32 + r32) * E_SROW + 2 * kh;
    const int b_off = 2 * E_AUNITS + (wn * 32 + r32) * E_SROW + 2 * kh;
    const uint32_t stride = (uint32_t)a.nch * (uint32_t)(E_UNITS * 16);

    // all loads of chunk ch: A rows into A stage ast, B columns into the B stage
    // (the last instruction only for the waves whose units lie inside the chunk)
    auto issue = [&](uint32_t ch, int ast) {
#pragma unroll
        for (int i = 0; i < E_LOADS; ++i) {
            const int first = i * E_THREADS + wave * 64;          // uniform per wave
            if (first >= E_UNITS_CHUNK) continue;
            const bool in_a = first < E_AUNITS;
            const int v = (in_a ? first : first - E_AUNITS) + lane;
            const int row = v / E_SROW, c = v % E_SROW;
            const uint32_t row0 = in_a ? (uint32_t)m0 : (uint32_t)n0;
            const uint8_t *src = (in_a ? a.QA : a.QB) +
                                 ((row0 + (uint32_t)row) * stride + ch * (uint32_t)(E_UNITS * 16) +
                                  (uint32_t)(c < E_UNITS ? c : E_UNITS - 1) * 16u);
            u32x4 *dst = in_a ? lds + ast * E_AUNITS + first : lds + 2 * E_AUNITS + (first - E_AUNITS);
            __builtin_amdgcn_global_load_lds((const void *)src,
                                             (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
        }
    };
    auto frag = [&](int off) {
        const v4i x0 = __builtin_bit_cast(v4i, lds[off]), x1 = __builtin_bit_cast(v4i, lds[off + 1]);
        return (v8i_t)__builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7);
    };

    v16f acc[11];
#pragma unroll
    for (int l = 0; l < 11; ++l) acc[l] = v16f{};
    // this lane's exact sums in the workspace: hi r at sums[r * 64], lo r at
    // sums[(16 + r) * 64] (lanes adjacent, so each access is one coalesced run)
    double *sums = a.sums + ((int64_t)blockIdx.x * 4 + wave) * 32 * 64 + lane;
#pragma unroll
    for (int r = 0; r < 32; ++r) sums[r * 64] = 0.0;

    // level lv (0-based: slices s + t = lv) into hi (lv <= 4, units of level 4) or
    // lo (units of level 10); both stay exact integers below 2^53 within a pass
    auto flush = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double hi = sums[r * 64], lo = sums[(16 + r) * 64];
#pragma unroll
            for (int lv = 0; lv < 11; ++lv) {
                const double sc = (double)(1 << (5 * (lv < 5 ? 4 - lv : 10 - lv)));
                if (lv < 5) hi = fma((double)acc[lv][r], sc, hi);
                else lo = fma((double)acc[lv][r], sc, lo);
            }
            sums[r * 64] = hi;
            sums[(16 + r) * 64] = lo;
        }
#pragma unroll
        for (int lv = 0; lv < 11; ++lv) acc[lv] = v16f{};
    };

    const uint32_t c0 = (uint32_t)a.ch0, c1 = (uint32_t)a.ch1;
    issue(c0, 0);
    for (uint32_t c = c0; c < c1; ++c) {
        const int ast = (int)((c - c0) & 1);
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));          // own loads of chunk c landed
        __syncthreads();                                  // everyone's
        v8i_t fb[11];
#pragma unroll
        for (int t = 0; t < 11; ++t) fb[t] = frag(b_off + 4 * t);
        __syncthreads();                                  // the B stage is free again
        if (c + 1 < c1) issue(c + 1, ast ^ 1);
        const int abase = ast * E_AUNITS + a_off;
        v8i_t fa = frag(abase);
#pragma unroll
        for (int s = 0; s < 11; ++s) {
            const v8i_t fcur = fa;
            if (s + 1 < 11) fa = frag(abase + 4 * (s + 1));
#pragma unroll
            for (int t = 0; t + s < 11; ++t)
                acc[s + t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    fcur, fb[t], acc[s + t], 0, 0, 0, 0, 0, 0);
        }
        if ((c - c0 + 1) % E_FLUSH == 0 || c + 1 == c1) flush();
    }
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));

    // exact value = hi 2^-28 + lo 2^-58, rounded once
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const double v = fma(sums[r * 64], 0x1p-28, sums[(16 + r) * 64] * 0x1p-58);
        store_c(a, m0 + wm * 32 + acc_row(lane, r), n0 + wn * 32 + r32, v);
    }
}

// ---------------------------------------------------------------------------
// Host side: workspace and driver.
// ---------------------------------------------------------------------------
constexpr int MAX_DEVICES = 64;

struct Workspace {
    std::mutex mtx;
    uint8_t *base = nullptr;
    size_t bytes = 0;
    int *host_flag = nullptr;        // pinned
    hipEvent_t done = nullptr;       // last split work that used the workspace
};

static Workspace g_ws[MAX_DEVICES];

// Marks the workspace in use until the work just queued on s has finished; if
// the event cannot be recorded, waits for that work instead.
static int32_t ws_mark(Workspace &w, hipStream_t s) {
    if (hipEventRecord(w.done, s) == hipSuccess) return 0;
    (void)hipGetLastError();
    const hipError_t he = hipStreamSynchronize(s);
    return he == hipSuccess ? 0 : set_error(MGEMM_ERR_HIP, "workspace: %s", hipGetErrorString(he));
}

static int32_t ws_reserve(Workspace &w, size_t bytes) {
    if (!w.done) {
        if (hipEventCreateWithFlags(&w.done, hipEventDisableTiming) != hipSuccess)
            return set_error(MGEMM_ERR_HIP, "split: event create failed");
    }
    if (!w.host_flag) {
        if (hipHostMalloc((void **)&w.host_flag, sizeof(int), hipHostMallocDefault) != hipSuccess)
            return set_error(MGEMM_ERR_NOMEM, "split: pinned flag allocation failed");
    }
    if (w.bytes >= bytes) return 0;
    if (w.base) {
        // the old buffer is freed only once its last user has finished
        const hipError_t he = hipEventSynchronize(w.done);
        if (he != hipSuccess)
            return set_error(MGEMM_ERR_HIP, "workspace: %s", hipGetErrorString(he));
        (void)hipFree(w.base);
        w.base = nullptr;
        w.bytes = 0;
    }
    if (hipMalloc((void **)&w.base, bytes) != hipSuccess) {
        (void)hipGetLastError();
        w.base = nullptr;
        return set_error(MGEMM_ERR_NOMEM, "split: workspace of %zu bytes not available", bytes);
    }
    w.bytes = bytes;
    return 0;
}

static inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// A slice-pair kernel and its launch shape.
struct PairKernel {
    void (*fn)(PairArgs);
    int tile_m, tile_n, threads;
    int kpad;         // k padded to a multiple of this (a multiple of KPAD)
    int chunk_mult;   // each pass covers a multiple of this many chunks
    bool sums = false;  // needs PairArgs::sums (16 bytes per element of C)
};

constexpr int64_t SPLIT_PAD = 128;   // m and n padded to a multiple of every pair tile

template <typename F>
static int32_t run_split(const GemmArgs &g, hipStream_t s, Workspace &w, int max_pass_k,
                         PairKernel pk) {
    const int64_t mp = round_up(g.m, SPLIT_PAD), np = round_up(g.n, SPLIT_PAD),
                  kp = round_up(g.k, pk.kpad);
    const size_t a_bytes = (size_t)mp * kp * F::S * F::ELEM;
    const size_t b_bytes = (size_t)np * kp * F::S * F::ELEM;
    const size_t e_bytes = round_up(mp * 4, 256), f_bytes = round_up(np * 4, 256);
    // the FP8 pair kernel keeps its exact sums (16 bytes per element of C) here
    const size_t s_bytes = pk.sums ? (size_t)mp * np * 16 : 0;
    const size_t total = e_bytes + f_bytes + 256 + a_bytes + b_bytes + s_bytes;
    int32_t rc = ws_reserve(w, total);
    if (rc) return rc;
    int *e = (int *)w.base;
    int *fexp = (int *)(w.base + e_bytes);
    int *flag = (int *)(w.base + e_bytes + f_bytes);
    uint8_t *QA = w.base + e_bytes + f_bytes + 256;
    uint8_t *QB = QA + a_bytes;
    double *sums = pk.sums ? (double *)(QB + b_bytes) : nullptr;

    hipError_t he = hipStreamWaitEvent(s, w.done, 0);
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "split: %s", hipGetErrorString(he));
    hipLaunchKernelGGL(split_init_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s,
                       fexp, np, flag);
    hipLaunchKernelGGL(split_row_scale_kernel, dim3((unsigned)(g.m < 65536 ? g.m : 65536)),
                       dim3(256), 0, s, (const double *)g.A, g.m, g.k, g.lda, e, flag);
    {
        int64_t gy = (g.k + COL_ROWS - 1) / COL_ROWS;
        if (gy > 65535) gy = 65535;
        hipLaunchKernelGGL(split_col_scale_kernel, dim3((unsigned)((g.n + 255) / 256), (unsigned)gy),
                           dim3(256), 0, s, (const double *)g.B, g.k, g.n, g.ldb, fexp, flag);
    }
    he = hipMemcpyAsync(w.host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "split scale: %s", hipGetErrorString(he));
    if (*w.host_flag) return set_error(MGEMM_ERR_NONFINITE, "split: A or B holds NaN or Inf");

    {
        int64_t groups = mp * (kp / 8);
        int64_t blocks = (groups + 255) / 256;
        if (blocks > 1 << 20) blocks = 1 << 20;
        hipLaunchKernelGGL(split_slice_a_kernel<F>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double *)g.A, g.m, g.k, g.lda, (const int *)e, QA, mp, kp);
        hipLaunchKernelGGL(split_slice_b_kernel<F>, dim3((unsigned)(np / 64), (unsigned)(kp / 64)),
                           dim3(256), 0, s, (const double *)g.B, g.k, g.n, g.ldb,
                           (const int *)fexp, QB, kp);
    }

    PairArgs pa;
    pa.QA = QA;
    pa.QB = QB;
    pa.e = e;
    pa.fexp = fexp;
    pa.C = (double *)g.C;
    pa.m = g.m;
    pa.n = g.n;
    pa.ldc = g.ldc;
    pa.nch = kp / F::KC;
    pa.alpha = g.alpha;
    pa.tiles_m = (int)(mp / pk.tile_m);
    pa.tiles_n = (int)(np / pk.tile_n);
    pa.sums = sums;
    const int64_t blocks = (int64_t)pa.tiles_m * pa.tiles_n;
    const int64_t pass_ch = max_pass_k / F::KC;
    // chunks holding data, rounded up to the kernel's multiple (zero slices)
    const int64_t kch = round_up((g.k + F::KC - 1) / F::KC, pk.chunk_mult);
    for (int64_t c0 = 0; c0 < kch; c0 += pass_ch) {
        pa.ch0 = c0;
        pa.ch1 = c0 + pass_ch < kch ? c0 + pass_ch : kch;
        pa.beta = c0 == 0 ? g.beta : 1.0;
        hipLaunchKernelGGL(pk.fn, dim3((unsigned)blocks), dim3(pk.threads), 0, s, pa);
    }
    he = hipGetLastError();
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "split launch: %s", hipGetErrorString(he));
    return ws_mark(w, s);
}

// Modular-integer emulation: the scale step above, then the residue, product and
// reconstruction kernels of crt.hip on the same workspace.
static int32_t run_crt(const GemmArgs &g, hipStream_t s, Workspace &w) {
    const int64_t mp = round_up(g.m, CRT_TILE), np = round_up(g.n, CRT_TILE),
                  kp = round_up(g.k, CRT_KSTEP);
    // the product kernel addresses a tile's rows of one plane with 32-bit offsets
    if ((double)CRT_TILE * (double)kp >= 4294967296.0)
        return set_error(MGEMM_ERR_NOCONFIG, "crt int8: k above 2^24 - 64");
    const size_t qa_bytes = (size_t)CRT_MODULI * mp * kp, qb_bytes = (size_t)CRT_MODULI * np * kp;
    const size_t r_bytes = (size_t)CRT_MODULI * mp * np;
    const size_t e_bytes = round_up(mp * 4, 256), f_bytes = round_up(np * 4, 256);
    int32_t rc = ws_reserve(w, e_bytes + f_bytes + 256 + qa_bytes + qb_bytes + r_bytes);
    if (rc) return rc;
    int *e = (int *)w.base;
    int *fexp = (int *)(w.base + e_bytes);
    int *flag = (int *)(w.base + e_bytes + f_bytes);
    int8_t *QA = (int8_t *)(w.base + e_bytes + f_bytes + 256);
    int8_t *QB = QA + qa_bytes;
    uint8_t *R = (uint8_t *)(QB + qb_bytes);

    hipError_t he = hipStreamWaitEvent(s, w.done, 0);
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "crt: %s", hipGetErrorString(he));
    hipLaunchKernelGGL(split_init_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s,
                       fexp, np, flag);
    hipLaunchKernelGGL(split_row_scale_kernel, dim3((unsigned)(g.m < 65536 ? g.m : 65536)),
                       dim3(256), 0, s, (const double *)g.A, g.m, g.k, g.lda, e, flag);
    {
        int64_t gy = (g.k + COL_ROWS - 1) / COL_ROWS;
        if (gy > 65535) gy = 65535;
        hipLaunchKernelGGL(split_col_scale_kernel, dim3((unsigned)((g.n + 255) / 256), (unsigned)gy),
                           dim3(256), 0, s, (const double *)g.B, g.k, g.n, g.ldb, fexp, flag);
    }
    he = hipMemcpyAsync(w.host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "crt scale: %s", hipGetErrorString(he));
    if (*w.host_flag) return set_error(MGEMM_ERR_NONFINITE, "crt: A or B holds NaN or Inf");

    he = crt_launch(g, s, e, fexp, crt_operand_bits(g.k), QA, QB, R, mp, np, kp);
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "crt launch: %s", hipGetErrorString(he));
    return ws_mark(w, s);
}

int32_t split_gemm(const GemmArgs &g, int32_t dtype, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return set_error(MGEMM_ERR_HIP, "split: no current device");
    Workspace &w = g_ws[dev];
    std::lock_guard<std::mutex> lock(w.mtx);
    if (dtype == MGEMM_SPLIT_BF16) {
        // the pipelined kernel addresses each operand's slices with 32-bit offsets;
        // larger operands take the register-staged kernel (64-bit addresses)
        const double big = (double)round_up(g.m > g.n ? g.m : g.n, SPLIT_PAD) *
                           (double)round_up(g.k, 256) * FmtBF16::S * FmtBF16::ELEM;
        if (big < 4294967296.0)
            return run_split<FmtBF16>(g, s, w, 1 << 17,
                                      PairKernel{split_pairs_bf16_pipe_kernel, R_BM, R_BN, R_THREADS,
                                                 256, R_BLOCK});
        return run_split<FmtBF16>(g, s, w, 1 << 17,
                                  PairKernel{split_pairs_bf16_kernel, PBM, PBN, 512, KPAD, 1});
    }
    if (dtype == MGEMM_SPLIT_INT8) {
        // the pipelined kernel addresses each operand's slices with 32-bit offsets
        const double big = (double)round_up(g.m > g.n ? g.m : g.n, SPLIT_PAD) *
                           (double)round_up(g.k, KPAD) * FmtI8::S;
        if (big >= 4294967296.0)
            return set_error(MGEMM_ERR_NOCONFIG, "split int8: slices of one operand exceed 4 GiB");
        return run_split<FmtI8>(g, s, w, 1 << 14,
                                PairKernel{split_pairs_i8_pipe_kernel, Q_BM, Q_BN, 256, KPAD, 1});
    }
    if (dtype == MGEMM_SPLIT_FP8) {
        // the pair kernel addresses each operand's slices with 32-bit offsets
        const double big = (double)round_up(g.m > g.n ? g.m : g.n, SPLIT_PAD) *
                           (double)round_up(g.k, KPAD) * FmtE4M3::S;
        if (big >= 4294967296.0)
            return set_error(MGEMM_ERR_NOCONFIG, "split fp8: slices of one operand exceed 4 GiB");
        return run_split<FmtE4M3>(g, s, w, 1 << 17,
                                  PairKernel{split_pairs_e4m3_kernel, E_BM, E_BN, E_THREADS, KPAD, 1,
                                             true});
    }
    if (dtype == MGEMM_CRT_INT8) return run_crt(g, s, w);
    return set_error(MGEMM_ERR_NOCONFIG, "split dtype %d is not built", dtype);
}

int32_t with_workspace(size_t bytes, hipStream_t s, const std::function<int32_t(uint8_t *)> &fn) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return set_error(MGEMM_ERR_HIP, "workspace: no current device");
    Workspace &w = g_ws[dev];
    std::lock_guard<std::mutex> lock(w.mtx);
    int32_t rc = ws_reserve(w, bytes);
    if (rc) return rc;
    hipError_t he = hipStreamWaitEvent(s, w.done, 0);
    if (he != hipSuccess) return set_error(MGEMM_ERR_HIP, "workspace: %s", hipGetErrorString(he));
    rc = fn(w.base);
    const int32_t mrc = ws_mark(w, s);
    return rc ? rc : mrc;
}

int32_t split_release() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 0;
    Workspace &w = g_ws[dev];
    std::lock_guard<std::mutex> lock(w.mtx);
    if (w.base) {
        const hipError_t he = hipEventSynchronize(w.done);
        if (he != hipSuccess)
            return set_error(MGEMM_ERR_HIP, "workspace release: %s", hipGetErrorString(he));
        (void)hipFree(w.base);
        w.base = nullptr;
        w.bytes = 0;
    }
    return 0;
}

}  // namespace mgemm

extern "C" int32_t mgemm_release_workspace(void) { return mgemm::split_release(); }
