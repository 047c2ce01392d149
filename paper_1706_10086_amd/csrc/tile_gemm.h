// The two-stage tiled GEMM of one C tile (tile_gemm), its single-GEMM kernel
// and launcher: shared by the hand-registered configurations (gemm_tiled.hip)
// and the tuning-grid configurations (grid_*.hip).
//
// The computation is the paper's tiled GEMM (Sec. 2.1, Fig. 2): a work-group owns
// one BM x BN tile of C, walks k in steps of BK staging one BM x BK tile of A and
// one BK x BN tile of B in LDS (the tile cache of Eq. 5), multiplies them into
// register sub-tiles of C on the matrix cores (the thread-local C tile of Fig. 2,
// the multiply-add of Listing 2) and streams C once at the end.
#pragma once

#include "mgemm_internal.h"

namespace mgemm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Pointer qualifier for global memory: loads and stores through it compile to
// global instructions, never to generic (flat) ones.
#define AS_GLOBAL __attribute__((address_space(1)))

// ---------------------------------------------------------------------------
// Element-type traits: vector types and the 16x16xK MFMA step.
// ---------------------------------------------------------------------------
template <typename T> struct Elem;

template <> struct Elem<double> {
    typedef v2d vec2;
    typedef v4d acc4;
    // D += A(16x4) * B(4x16); lane l supplies A[l%16][l/16] and B[l/16][l%16].
    __device__ static inline acc4 mma(double a, double b, acc4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // Row of D held in accumulator element r by lanes 16q..16q+15 (column l%16):
    // the FP64 instruction interleaves rows q, q+4, q+8, q+12.
    __device__ static inline int out_row(int q, int r) { return q + 4 * r; }
};

template <> struct Elem<float> {
    typedef v2f vec2;
    typedef v4f acc4;
    __device__ static inline acc4 mma(float a, float b, acc4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // The FP32 instruction gives lanes 16q..16q+15 the four rows 4q..4q+3.
    __device__ static inline int out_row(int q, int r) { return 4 * q + r; }
};

// alpha*acc + beta*c with each product and the sum rounded separately (no
// contraction into a fused multiply-add), the rounding of the definition.
template <typename T>
__device__ inline T scale_add(T alpha, T acc, T beta, T c) {
#pragma clang fp contract(off)
    return alpha * acc + beta * c;
}

// ---------------------------------------------------------------------------
// The kernel.
// ---------------------------------------------------------------------------
// T      element type (double or float)
// BM,BN  C tile of the work-group; BK depth of one k-step
// WGM,WGN waves along M and N (WGM*WGN waves, 64 lanes each)
// EPT    consecutive elements one thread copies per run (a multiple of 2)
// DBUF   two LDS stages (1) or one (0)
// ALIGN  A and B rows start on 2-element boundaries (even leading dimensions and
//        aligned base pointers): full runs use 2-element vector loads; otherwise
//        every element is loaded alone.
template <typename T, int BM, int BN, int BK, int DBUF>
struct TileLds {
    static constexpr int SA = BK + 2;                               // A row stride
    static constexpr int SB = BN + (sizeof(T) == 8 ? 8 : 16);       // B row stride
    static constexpr int STAGES = DBUF ? 2 : 1;
    static constexpr int A_ELEMS = STAGES * BM * SA;
    static constexpr int B_ELEMS = STAGES * BK * SB;
};

// One BM x BN tile of C at (m0, n0): the whole k-loop and the epilogue.  sAbase
// and sBbase are the work-group's LDS stages (TileLds sizes); the function ends
// with a barrier after the last read of LDS, so a caller may reuse the stages
// for another tile right away.
// SKIP_DEAD: on edge tiles a wave whose part of the tile lies wholly outside C
// runs no matrix-core steps (it still loads and stores its share of the LDS
// tiles; its results are never stored, and every stored sum is unchanged).
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, bool ALIGN,
          bool SKIP_DEAD = false>
__device__ __forceinline__ void tile_gemm(const GemmArgs &p, int64_t m0, int64_t n0, T *sAbase,
                                          T *sBbase) {
    typedef Elem<T> E;
    typedef typename E::vec2 vec2;
    typedef typename E::acc4 acc4;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WM = BM / WGM;           // C rows per wave
    constexpr int WN = BN / WGN;           // C columns per wave
    constexpr int FM = WM / 16;            // MFMA fragments per wave along M
    constexpr int FN = WN / 16;            // ... along N
    constexpr int SA = BK + 2;             // LDS row stride of the A tile (elements)
    constexpr int SB = BN + (sizeof(T) == 8 ? 8 : 16);  // LDS row stride of the B tile
    constexpr int STAGES = DBUF ? 2 : 1;
    constexpr int A_RUNS = BM * BK / (EPT * NT);   // runs per thread per k-step
    constexpr int B_RUNS = BK * BN / (EPT * NT);
    constexpr int A_RUNS_PER_ROW = BK / EPT;
    constexpr int B_RUNS_PER_ROW = BN / EPT;
    static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
    static_assert(BK % 8 == 0, "BK must be a multiple of 8");
    static_assert(EPT % 2 == 0, "EPT must be even");
    static_assert(A_RUNS >= 1 && A_RUNS * EPT * NT == BM * BK, "A tile split");
    static_assert(B_RUNS >= 1 && B_RUNS * EPT * NT == BK * BN, "B tile split");
    static_assert(A_RUNS_PER_ROW >= 1 && B_RUNS_PER_ROW >= 1, "EPT wider than a tile row");

    T (*sA)[BM * SA] = reinterpret_cast<T (*)[BM * SA]>(sAbase);
    T (*sB)[BK * SB] = reinterpret_cast<T (*)[BK * SB]>(sBbase);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WGN;             // wave position in the work-group grid
    const int wn = wave % WGN;

    // global address space: the operands of a batched problem come from a
    // descriptor in memory, and generic (flat) loads would also count against the
    // LDS wait counter, tying each LDS read to the outstanding prefetch
    const AS_GLOBAL T *__restrict__ A = (const AS_GLOBAL T *)p.A;
    const AS_GLOBAL T *__restrict__ B = (const AS_GLOBAL T *)p.B;
    AS_GLOBAL T *__restrict__ C = (AS_GLOBAL T *)p.C;
    const int64_t lda = p.lda, ldb = p.ldb, ldc = p.ldc;
    const int64_t mrem = p.m - m0;          // valid rows of this tile (may exceed BM)
    const int64_t nrem = p.n - n0;

    // Per-thread coordinates of its runs inside the A and B tiles.
    int a_row[A_RUNS], a_col[A_RUNS];
#pragma unroll
    for (int r = 0; r < A_RUNS; ++r) {
        int run = tid + r * NT;
        a_row[r] = run / A_RUNS_PER_ROW;
        a_col[r] = (run % A_RUNS_PER_ROW) * EPT;
    }
    int b_row[B_RUNS], b_col[B_RUNS];
#pragma unroll
    for (int r = 0; r < B_RUNS; ++r) {
        int run = tid + r * NT;
        b_row[r] = run / B_RUNS_PER_ROW;
        b_col[r] = (run % B_RUNS_PER_ROW) * EPT;
    }

    vec2 ra[A_RUNS][EPT / 2];
    vec2 rb[B_RUNS][EPT / 2];

    // Global -> registers for k-step starting at k0 (zero outside the matrix).
    auto load_tiles = [&](int64_t k0) {
        const int64_t krem = p.k - k0;
#pragma unroll
        for (int r = 0; r < A_RUNS; ++r) {
            const bool rok = a_row[r] < mrem;
            const AS_GLOBAL T *src = A + (m0 + a_row[r]) * lda + k0 + a_col[r];
#pragma unroll
            for (int v = 0; v < EPT / 2; ++v) {
                const int c = a_col[r] + 2 * v;
                vec2 x = {T(0), T(0)};
                if (rok) {
                    if (ALIGN && c + 1 < krem) {
                        x = *(const AS_GLOBAL vec2 *)(src + 2 * v);
                    } else {
                        if (c < krem) x[0] = src[2 * v];
                        if (c + 1 < krem) x[1] = src[2 * v + 1];
                    }
                }
                ra[r][v] = x;
            }
        }
#pragma unroll
        for (int r = 0; r < B_RUNS; ++r) {
            const bool rok = b_row[r] < krem;
            const AS_GLOBAL T *src = B + (k0 + b_row[r]) * ldb + n0 + b_col[r];
#pragma unroll
            for (int v = 0; v < EPT / 2; ++v) {
                const int c = b_col[r] + 2 * v;
                vec2 x = {T(0), T(0)};
                if (rok) {
                    if (ALIGN && c + 1 < nrem) {
                        x = *(const AS_GLOBAL vec2 *)(src + 2 * v);
                    } else {
                        if (c < nrem) x[0] = src[2 * v];
                        if (c + 1 < nrem) x[1] = src[2 * v + 1];
                    }
                }
                rb[r][v] = x;
            }
        }
    };

    auto store_tiles = [&](int st) {
#pragma unroll
        for (int r = 0; r < A_RUNS; ++r)
#pragma unroll
            for (int v = 0; v < EPT / 2; ++v)
                *(vec2 *)&sA[st][a_row[r] * SA + a_col[r] + 2 * v] = ra[r][v];
#pragma unroll
        for (int r = 0; r < B_RUNS; ++r)
#pragma unroll
            for (int v = 0; v < EPT / 2; ++v)
                *(vec2 *)&sB[st][b_row[r] * SB + b_col[r] + 2 * v] = rb[r][v];
    };

    acc4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc4{0, 0, 0, 0};

    const int l16 = lane & 15;     // row of A / column of B inside a fragment
    const int kq = lane >> 4;      // which pair of k values this lane feeds
    const int a_base = (wm * WM + l16) * SA + 2 * kq;
    const int b_base = (2 * kq) * SB + wn * WN + l16;

    auto multiply = [&](int st) {
        const T *tA = sA[st];
        const T *tB = sB[st];
#pragma unroll
        for (int g = 0; g < BK / 8; ++g) {
            vec2 af[FM];
            T bf0[FN], bf1[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                af[i] = *(const vec2 *)&tA[a_base + i * 16 * SA + g * 8];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                bf0[j] = tB[b_base + (g * 8) * SB + j * 16];
                bf1[j] = tB[b_base + (g * 8 + 1) * SB + j * 16];
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    acc[i][j] = E::mma(af[i][0], bf0[j], acc[i][j]);
                    acc[i][j] = E::mma(af[i][1], bf1[j], acc[i][j]);
                }
        }
    };

    // whether any row and column of this wave's part of the tile lie inside C
    // (uniform per wave)
    bool live = true;
    if (SKIP_DEAD)
        live = mrem > (int64_t)__builtin_amdgcn_readfirstlane(wm) * WM &&
               nrem > (int64_t)__builtin_amdgcn_readfirstlane(wn) * WN;

    const int64_t nk = (p.k + BK - 1) / BK;
    load_tiles(0);
    store_tiles(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = DBUF ? (int)(kt & 1) : 0;
        const bool more = kt + 1 < nk;
        if (more) load_tiles((kt + 1) * BK);
        if (live) multiply(cur);
        if (more) {
            if (!DBUF) __syncthreads();
            store_tiles(DBUF ? cur ^ 1 : 0);
        }
        __syncthreads();
    }

    // Epilogue: lane holds column l16 and rows E::out_row(kq, 0..3) of each fragment.
    // With small wave tiles (at most 8 fragments, registers to spare) interior tiles
    // issue all C loads of one fragment row before the stores (no per-element
    // bounds tests between them); otherwise, and on edge tiles, each element is
    // tested, loaded and stored in turn.
    const T alpha = (T)p.alpha;
    const T beta = (T)p.beta;
    const bool read_c = p.beta != 0.0;
    if (FM * FN <= 8 && mrem >= BM && nrem >= BN) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            T cv[FN][4];
            if (read_c) {
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        cv[j][r] = C[(m0 + wm * WM + i * 16 + E::out_row(kq, r)) * ldc + n0 +
                                     wn * WN + j * 16 + l16];
            }
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    AS_GLOBAL T *c = C + (m0 + wm * WM + i * 16 + E::out_row(kq, r)) * ldc + n0 + wn * WN +
                           j * 16 + l16;
                    *c = read_c ? scale_add(alpha, acc[i][j][r], beta, cv[j][r]) : alpha * acc[i][j][r];
                }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t col = wn * WN + j * 16 + l16;
            if (col >= nrem) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = wm * WM + i * 16 + E::out_row(kq, r);
                if (row >= mrem) continue;
                AS_GLOBAL T *c = C + (m0 + row) * ldc + n0 + col;
                *c = read_c ? scale_add(alpha, acc[i][j][r], beta, *c) : alpha * acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------------------
// Occupancy: the paper's hardware threads per core (Sec. 3, Tab. 4) as waves
// per SIMD.  OCC = o > 0 makes a kernel run at most o waves per SIMD: it is
// compiled for at least o waves per SIMD (registers <= 512 / o per lane), and its
// work-group allocates at least occupancy_lds_floor bytes of LDS, more than
// 1 / (g + 1) of the compute unit's 160 KiB, so that at most g = max(1,
// 4 o / waves) work-groups (o waves on each of the 4 SIMDs) share a compute unit.
// OCC = 0 leaves both to the compiler and the resources the kernel needs.
// ---------------------------------------------------------------------------
constexpr int LDS_PER_CU = 160 * 1024;

constexpr int occupancy_groups(int occ, int waves) {
    return 4 * occ / waves > 0 ? 4 * occ / waves : 1;
}

constexpr int occupancy_lds_floor(int occ, int waves) {
    return occ <= 0 ? 0 : LDS_PER_CU / (occupancy_groups(occ, waves) + 1) + 16;
}

// Elements of T to add to a work-group's natural LDS bytes to reach the floor.
template <typename T>
constexpr int occupancy_pad_elems(int occ, int waves, int natural_bytes) {
    return occupancy_lds_floor(occ, waves) > natural_bytes
               ? (occupancy_lds_floor(occ, waves) - natural_bytes + (int)sizeof(T) - 1) /
                     (int)sizeof(T)
               : 0;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
// OCC    waves per SIMD (see above; 0: no limit)

// One GEMM: one work-group per C tile.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC,
          bool ALIGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1)))
gemm_tiled_kernel(GemmArgs p) {
    typedef TileLds<T, BM, BN, BK, DBUF> L;
    constexpr int PAD = occupancy_pad_elems<T>(OCC, WGM * WGN,
                                               (L::A_ELEMS + L::B_ELEMS) * (int)sizeof(T));
    __shared__ __attribute__((aligned(16))) T sA[L::A_ELEMS + PAD];
    __shared__ __attribute__((aligned(16))) T sB[L::B_ELEMS];
    const int tiles_m = (int)((p.m + BM - 1) / BM);
    const int tiles_n = (int)((p.n + BN - 1) / BN);
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    tile_gemm<T, BM, BN, BK, WGM, WGN, EPT, DBUF, ALIGN>(p, (int64_t)tm * BM, (int64_t)tn * BN,
                                                          sA, sB);
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC,
          bool ALIGN>
hipError_t launch_tiled(const GemmArgs &a, hipStream_t s) {
    int64_t blocks = ((a.m + BM - 1) / BM) * ((a.n + BN - 1) / BN);
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((gemm_tiled_kernel<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, ALIGN>),
                       dim3((unsigned)blocks), dim3(64 * WGM * WGN), 0, s, a);
    return hipGetLastError();
}

}  // namespace mgemm
