// Tiled GEMM C = alpha*A*B + beta*C on gfx950 matrix cores, FP64 and FP32.
//
// The computation is the paper's tiled GEMM (Sec. 2.1, Fig. 2): each work-group
// owns one tile of C (Sec. 2.1: one C tile per block, the grid of Eq. 3 becoming
// ceil(m/BM) x ceil(n/BN) work-groups); an outer loop walks the k-dimension in
// steps of BK, staging one BM x BK tile of A and one BK x BN tile of B in LDS (the
// tile cache of Eq. 5, here (BM*BK + BK*BN) * S bytes per stage); an inner loop
// multiplies the staged tiles into a per-thread register sub-tile of C (the
// thread-local temporary C tile of Fig. 2, the multiply-add of Listing 2); C is
// read and written once at the end (the streamed epilogue of Fig. 2).
//
// gfx950 specifics (not from the paper):
//  * the inner multiply runs on MFMA: v_mfma_f64_16x16x4_f64 for FP64 and
//    v_mfma_f32_16x16x4_f32 for FP32, each wave owning a WM x WN block of C held
//    as (WM/16) x (WN/16) accumulator fragments;
//  * one lane of an MFMA fragment reads two consecutive k values of A with one
//    16-byte LDS read and feeds them to two MFMAs; B supplies the same two k rows,
//    so the k-sum is complete, only reordered;
//  * LDS rows are padded so the fragment reads are free of bank conflicts;
//  * global loads are coalesced runs of EPT consecutive elements per thread, and
//    with double buffering the next k-step's loads are in flight while the
//    current step is multiplied;
//  * work-group ids are remapped so that the work-groups placed on one XCD (the
//    hardware deals ids round-robin over the 8 XCDs) own a compact group of C
//    tiles and share their A and B panels in that XCD's L2.
#include <algorithm>
#include <vector>

#include "grid_registry.h"
#include "tile_gemm.h"

namespace mgemm {

// Many GEMMs sharing one configuration: a persistent grid whose work-groups take
// work items from atomic counters until every list is exhausted.  With a tile
// map (item = map entry: problem, tile row, tile column) there is one list per
// XCD, each holding whole problems or runs of a problem's tiles, so the panels of
// A and B that a run of tiles shares stay in that XCD's L2; a work-group drains
// its own XCD's list, then takes from the others.  Without a map the single list
// holds tile numbers (problems numbered tile by tile, BatchProblem::tile0 the
// first of each) and a tile's problem is found by binary search.  Lists order
// their problems by decreasing work.  Thread 0 asks for the next item as the
// work-group starts a tile, so the atomic's latency hides behind the tile's work.
// Split-k partial products: work-group (x, y) computes C tile x over the y-th
// range of kc values of k (columns of A, rows of B) with alpha = 1 and beta = 0,
// into plane y of W (m x n, row stride n); splitk_reduce_kernel sums the planes.
// A range starts at a multiple of kc (a multiple of BK), so rows keep the
// alignment of A and B.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC,
          bool ALIGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1)))
gemm_splitk_kernel(GemmArgs p, int64_t kc, T *W) {
    typedef TileLds<T, BM, BN, BK, DBUF> L;
    constexpr int PAD = occupancy_pad_elems<T>(OCC, WGM * WGN,
                                               (L::A_ELEMS + L::B_ELEMS) * (int)sizeof(T));
    __shared__ __attribute__((aligned(16))) T sA[L::A_ELEMS + PAD];
    __shared__ __attribute__((aligned(16))) T sB[L::B_ELEMS];
    const int tiles_m = (int)((p.m + BM - 1) / BM);
    const int tiles_n = (int)((p.n + BN - 1) / BN);
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t y = blockIdx.y, k0 = y * kc;
    GemmArgs q = p;
    q.k = p.k - k0 < kc ? p.k - k0 : kc;
    q.A = (const T *)p.A + k0;
    q.B = (const T *)p.B + k0 * p.ldb;
    q.alpha = 1.0;
    q.beta = 0.0;
    q.C = W + y * p.m * p.n;
    q.ldc = p.n;
    tile_gemm<T, BM, BN, BK, WGM, WGN, EPT, DBUF, ALIGN>(q, (int64_t)tm * BM, (int64_t)tn * BN,
                                                          sA, sB);
}

// C = alpha * (W_0 + W_1 + ... + W_{S-1}) + beta * C, the planes added in order
// (the same rounding of alpha and beta as the tile epilogue).  Rows run over
// blockIdx.y, columns over blockIdx.x and the threads (coalesced).
template <typename T>
__global__ void __launch_bounds__(256)
splitk_reduce_kernel(const T *__restrict__ W, int S, int64_t m, int64_t n, T alpha, T beta,
                     int read_c, T *C, int64_t ldc) {
    const int64_t plane = m * n;
    for (int64_t row = blockIdx.y; row < m; row += gridDim.y)
        for (int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x; col < n;
             col += (int64_t)gridDim.x * 256) {
            const int64_t i = row * n + col;
            T acc = W[i];
            for (int y = 1; y < S; ++y) acc += W[y * plane + i];
            T *c = C + row * ldc + col;
            *c = read_c ? scale_add(alpha, acc, beta, *c) : alpha * acc;
        }
}

// Waves per SIMD the batched kernel is compiled for: the configuration's
// occupancy if it names one; for the four-wave 64 x 64 x 16 tile three (it
// still fits without spilling, and a batch of short tiles is bound by load
// latency, which more resident work-groups hide; FP64 spills at four, FP32 fits
// four but ran no faster).
constexpr int batched_waves(int bm, int bn, int bk, int waves, int occ) {
    return occ > 0 ? occ : (bm * bn <= 64 * 64 && bk <= 16 && waves == 4 ? 3 : 1);
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC>
__global__ void __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(batched_waves(BM, BN, BK, WGM * WGN, OCC))))
gemm_batched_kernel(const BatchProblem *__restrict__ probs, const uint64_t *__restrict__ tile_map,
                    const int64_t *__restrict__ list_off, int nlist, int nprob,
                    unsigned long long *counters) {
    typedef TileLds<T, BM, BN, BK, DBUF> L;
    __shared__ __attribute__((aligned(16))) T sA[L::A_ELEMS];
    __shared__ __attribute__((aligned(16))) T sB[L::B_ELEMS];
    __shared__ int64_t next;
    // the item index is uniform: keep it (and all that follows from it) in
    // scalar registers
    auto uniform_next = [&]() {
        const uint64_t tv = (uint64_t)next;
        return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(tv >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)tv));
    };
    // thread 0's state: lists visited so far and the counter value last taken
    const int home = (int)(blockIdx.x % (unsigned)nlist);
    int visit = 0;
    unsigned long long taken = 0;
    // (thread 0) the item that `taken` names, moving on to the next list while
    // the current one is exhausted; -1 once every list is
    auto settle = [&]() -> int64_t {
        for (;;) {
            const int l = home + visit < nlist ? home + visit : home + visit - nlist;
            const int64_t idx = list_off[l] + (int64_t)taken;
            if (idx < list_off[l + 1]) return idx;
            if (++visit >= nlist) return -1;
            const int l2 = home + visit < nlist ? home + visit : home + visit - nlist;
            taken = atomicAdd(&counters[l2], 1ull);
        }
    };
    if (threadIdx.x == 0) {
        taken = atomicAdd(&counters[home], 1ull);
        next = settle();
    }
    __syncthreads();
    int64_t t = uniform_next();
    while (t >= 0) {
        if (threadIdx.x == 0) {
            const int l = home + visit < nlist ? home + visit : home + visit - nlist;
            taken = atomicAdd(&counters[l], 1ull);                // read after this tile
        }
        int pi;
        int64_t tm, tn;
        if (tile_map) {
            const uint64_t e = tile_map[t];
            const uint64_t eu = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(e >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)e);
            constexpr uint64_t RC = (1ull << TILE_MAP_RC_BITS) - 1;
            pi = (int)(eu >> (2 * TILE_MAP_RC_BITS));
            tm = (int64_t)((eu >> TILE_MAP_RC_BITS) & RC);
            tn = (int64_t)(eu & RC);
        } else {
            int lo = 0, hi = nprob - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (probs[mid].tile0 <= t) lo = mid;
                else hi = mid - 1;
            }
            pi = lo;
            tm = tn = -1;
        }
        // copy the (uniform) descriptor word by word into scalar registers
        BatchProblem bp;
        {
            const uint32_t *src = reinterpret_cast<const uint32_t *>(probs + pi);
            uint32_t *dst = reinterpret_cast<uint32_t *>(&bp);
#pragma unroll
            for (int w = 0; w < (int)(sizeof(BatchProblem) / 4); ++w)
                dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
        }
        if (tm < 0) {
            const int64_t local = t - bp.tile0;
            tm = local / bp.tiles_n;
            tn = local - tm * bp.tiles_n;
        }
        // the tile runs gemm_ex's code for its problem's row alignment
        if (bp.aligned)
            tile_gemm<T, BM, BN, BK, WGM, WGN, EPT, DBUF, true, true>(bp.g, tm * BM, tn * BN, sA, sB);
        else
            tile_gemm<T, BM, BN, BK, WGM, WGN, EPT, DBUF, false, true>(bp.g, tm * BM, tn * BN, sA,
                                                                        sB);
        __syncthreads();                  // every wave has read the current index
        if (threadIdx.x == 0) next = settle();
        __syncthreads();
        t = uniform_next();
    }
}

// ---------------------------------------------------------------------------
// Pipelined single-GEMM kernel: three LDS stages, direct global->LDS loads.
// ---------------------------------------------------------------------------
// WGM x WGN waves (4 or 8: one or two per SIMD), each owning a WM x WN block of
// C as (WM/16) x (WN/16) accumulator fragments.  Each k-step's A and B tiles are
// copied into LDS by global_load_lds (16 bytes per lane, no staging registers);
// while the products of k-step c run from registers, every fragment register is
// refilled with k-step c+1 right after its last use, and k-step c+2 is loading
// into the third stage, so the one barrier per k-step publishes a stage whose
// loads were issued a whole k-step earlier.  The k-sum order per element is the
// same as gemm_tiled_kernel's, so both give bit-identical results.
//
// Requirements (checked by the launcher, which otherwise runs the two-stage
// kernel of the same tile): n, lda and ldb even, A and B 16-byte aligned.  A
// partial last k-step (k not a multiple of BK) is loaded element-wise and
// zero-padded after the pipelined loop.  Rows >= m and columns >= n of the edge
// tiles load clamped (valid) addresses; their products only reach outputs that
// are not stored.
template <typename T, int BM, int BN, int BK, int WGM, int WGN>
struct PipeShape {
    static constexpr int NT = 64 * WGM * WGN;
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int FM = WM / 16, FN = WN / 16;
    static constexpr int G = BK / 8;                               // 8-deep k groups
    static constexpr int ROW_A = BK * (int)sizeof(T) / 16;         // 16-byte units per A row
    static constexpr int AU = ROW_A + 1;                           // padded A row (units)
    static constexpr int ROW_B = BN * (int)sizeof(T) / 16;         // units per B row
    // padded B row: stride BN + 8 elements, so the two k rows (2 kq apart) one
    // fragment read touches fall in distinct banks
    static constexpr int BU = ROW_B + (sizeof(T) == 8 ? 4 : 2);
    static constexpr int A_UNITS = BM * AU;
    static constexpr int STAGE = A_UNITS + BK * BU;                // units per stage
    static constexpr int LOADS = (STAGE + NT - 1) / NT;            // load instructions per wave
    static constexpr int EPU = 16 / (int)sizeof(T);                // elements per unit
};

// One BM x BN tile (tm, tn) of C: the three-stage k-loop and the epilogue; lds
// holds the three stages.
template <typename T, int BM, int BN, int BK, int WGM, int WGN>
__device__ __forceinline__ void pipe_tile(const GemmArgs &p, u32x4_t *lds, int tm, int tn) {
    typedef PipeShape<T, BM, BN, BK, WGM, WGN> S;
    typedef Elem<T> E;
    typedef typename E::vec2 vec2;
    typedef typename E::acc4 acc4;
    static_assert(S::WM % 16 == 0 && S::WN % 16 == 0 && BK % 8 == 0, "tile shape");

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WGN, wn = wave % WGN;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const T *__restrict__ A = (const T *)p.A;
    const T *__restrict__ B = (const T *)p.B;
    const int64_t lda = p.lda, ldb = p.ldb;

    // Per-lane source byte offsets of each load instruction, relative to the
    // tile's A panel (A + m0*lda) or B panel (B + n0) at k-step 0.  A wave's 64
    // units of one instruction lie in one region (A_UNITS is a multiple of 64), so
    // the panel address is wave-uniform and each load takes one offset register.
    static_assert(S::A_UNITS % 64 == 0, "A region must end on a wave's load");
    uint32_t src_off[S::LOADS];
#pragma unroll
    for (int i = 0; i < S::LOADS; ++i) {
        const int u = i * S::NT + wave * 64 + lane;
        int64_t e;
        if (u < S::A_UNITS) {
            const int r = u / S::AU, c = u % S::AU;
            const int64_t row = m0 + r < p.m ? r : p.m - 1 - m0;
            e = row * lda + (c < S::ROW_A ? c : S::ROW_A - 1) * S::EPU;
        } else {
            const int v = u - S::A_UNITS;
            const int r = v / S::BU, c = v % S::BU;
            int64_t col = (int64_t)(c < S::ROW_B ? c : S::ROW_B - 1) * S::EPU;
            if (col > p.n - n0 - S::EPU) col = p.n - n0 - S::EPU;
            e = (int64_t)(r < BK ? r : BK - 1) * ldb + col;
        }
        src_off[i] = (uint32_t)(e * (int64_t)sizeof(T));
    }
    const char *Apanel = (const char *)(A + m0 * lda);
    const char *Bpanel = (const char *)(B + n0);
    // load instruction i of k-step kstep into stage
    auto issue_one = [&](int i, int64_t kstep, u32x4_t *stage) {
        const int first = i * S::NT + wave * 64;
        // only the last instruction can run past the stage (uniform per wave)
        if ((i + 1) * S::NT > S::STAGE && first >= S::STAGE) return;
        const char *src = first < S::A_UNITS ? Apanel + kstep * (BK * (int64_t)sizeof(T))
                                             : Bpanel + kstep * (BK * ldb * (int64_t)sizeof(T));
        __builtin_amdgcn_global_load_lds((const void *)(src + src_off[i]),
                                         (__attribute__((address_space(3))) void *)(stage + first),
                                         16, 0, 0);
    };
    auto issue = [&](int64_t kstep, u32x4_t *stage) {
#pragma unroll
        for (int i = 0; i < S::LOADS; ++i) issue_one(i, kstep, stage);
    };

    acc4 acc[S::FM][S::FN];
#pragma unroll
    for (int i = 0; i < S::FM; ++i)
#pragma unroll
        for (int j = 0; j < S::FN; ++j) acc[i][j] = acc4{0, 0, 0, 0};

    const int l16 = lane & 15, kq = lane >> 4;
    // A fragment (g, i): elements g*8 + 2kq, +1 of row wm*WM + i*16 + l16; B fragment
    // (g, h, j): element (g*8 + 2kq + h, wn*WN + j*16 + l16) of the B region
    const int a_elem = (wm * S::WM + l16) * S::AU * S::EPU + 2 * kq;
    const int b_elem = S::A_UNITS * S::EPU + (2 * kq) * S::BU * S::EPU + wn * S::WN + l16;
    vec2 af[S::G][S::FM];
    T bf[S::G][2][S::FN];
    auto read_a = [&](const u32x4_t *st, int g, int i) {
        af[g][i] = *(const vec2 *)((const T *)st + a_elem + i * 16 * S::AU * S::EPU + g * 8);
    };
    auto read_b = [&](const u32x4_t *st, int g, int h) {
        const T *stT = (const T *)st;
#pragma unroll
        for (int j = 0; j < S::FN; ++j)
            bf[g][h][j] = stT[b_elem + (g * 8 + h) * S::BU * S::EPU + j * 16];
    };
    // products of one k-step; each fragment is refilled from the next stage right
    // after its last use (past the last k-step the refills read a stale stage and
    // are never used)
    // The k-step's loads (k-step lk into stage lst) are spread over the products,
    // one every few fragment rows, so the memory pipeline takes a few at a time
    // instead of every wave queueing all of them at the barrier.
    auto products = [&](const u32x4_t *nst, int64_t lk, u32x4_t *lst) {
        constexpr int SLOTS = S::G * 2 * S::FM;
        constexpr int EVERY = SLOTS / S::LOADS > 0 ? SLOTS / S::LOADS : 1;
        static_assert((S::LOADS - 1) * EVERY < SLOTS, "every load gets a slot");
#pragma unroll
        for (int g = 0; g < S::G; ++g) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int i = 0; i < S::FM; ++i) {
#pragma unroll
                    for (int j = 0; j < S::FN; ++j)
                        acc[i][j] = E::mma(af[g][i][h], bf[g][h][j], acc[i][j]);
                    if (h == 1) read_a(nst, g, i);
                    const int slot = (g * 2 + h) * S::FM + i;
                    if (slot % EVERY == 0 && slot / EVERY < S::LOADS) issue_one(slot / EVERY, lk, lst);
                    if (h == 1 || slot % EVERY == 0) __builtin_amdgcn_sched_barrier(0);
                }
                read_b(nst, g, h);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    const int64_t nk = p.k / BK;                 // full k-steps
    const int ktail = (int)(p.k % BK);           // depth of the partial last k-step
    if (nk > 0) {
        issue(0, lds);
        issue(nk > 1 ? 1 : 0, lds + S::STAGE);
        __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0)
        __syncthreads();
#pragma unroll
        for (int g = 0; g < S::G; ++g) {
#pragma unroll
            for (int i = 0; i < S::FM; ++i) read_a(lds, g, i);
            read_b(lds, g, 0);
            read_b(lds, g, 1);
        }
        // Past the end the loads repeat the last k-step (in bounds, never used),
        // which keeps the loop free of branches around the products.
        int st = 0;
        for (int64_t c = 0; c < nk; ++c) {
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): own loads of k-step c+1
            __syncthreads();
            const int st1 = st == 2 ? 0 : st + 1;
            const int st2 = st1 == 2 ? 0 : st1 + 1;
            products(lds + st1 * S::STAGE, c + 2 < nk ? c + 2 : nk - 1, lds + st2 * S::STAGE);
            st = st1;
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);      // no load may land after this point
    }
    if (ktail) {
        // The partial k-step: element-wise loads, zero outside A and B (as the
        // two-stage kernel pads), into stage 0 once every wave is done with LDS.
        __syncthreads();
        const int64_t k0 = nk * BK;
        T *sT = (T *)lds;
        for (int e = tid; e < BM * BK; e += S::NT) {
            const int r = e / BK, c = e % BK;
            sT[r * S::AU * S::EPU + c] =
                m0 + r < p.m && c < ktail ? A[(m0 + r) * lda + k0 + c] : (T)0;
        }
        for (int e = tid; e < BK * BN; e += S::NT) {
            const int r = e / BN, c = e % BN;
            sT[S::A_UNITS * S::EPU + r * S::BU * S::EPU + c] =
                r < ktail && n0 + c < p.n ? B[(k0 + r) * ldb + n0 + c] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < S::G; ++g) {
#pragma unroll
            for (int i = 0; i < S::FM; ++i) read_a(lds, g, i);
            read_b(lds, g, 0);
            read_b(lds, g, 1);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < S::FM; ++i)
#pragma unroll
                    for (int j = 0; j < S::FN; ++j)
                        acc[i][j] = E::mma(af[g][i][h], bf[g][h][j], acc[i][j]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // Epilogue as in tile_gemm: batched C loads for interior tiles.
    T *__restrict__ C = (T *)p.C;
    const int64_t ldc = p.ldc, mrem = p.m - m0, nrem = p.n - n0;
    const T alpha = (T)p.alpha, beta = (T)p.beta;
    const bool read_c = p.beta != 0.0;
    if (mrem >= BM && nrem >= BN) {
#pragma unroll
        for (int i = 0; i < S::FM; ++i) {
            T cv[S::FN][4];
            if (read_c) {
#pragma unroll
                for (int j = 0; j < S::FN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        cv[j][r] = C[(m0 + wm * S::WM + i * 16 + E::out_row(kq, r)) * ldc + n0 +
                                     wn * S::WN + j * 16 + l16];
            }
#pragma unroll
            for (int j = 0; j < S::FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T *c = C + (m0 + wm * S::WM + i * 16 + E::out_row(kq, r)) * ldc + n0 +
                           wn * S::WN + j * 16 + l16;
                    *c = read_c ? scale_add(alpha, acc[i][j][r], beta, cv[j][r]) : alpha * acc[i][j][r];
                }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < S::FM; ++i)
#pragma unroll
        for (int j = 0; j < S::FN; ++j) {
            const int64_t col = wn * S::WN + j * 16 + l16;
            if (col >= nrem) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = wm * S::WM + i * 16 + E::out_row(kq, r);
                if (row >= mrem) continue;
                T *c = C + (m0 + row) * ldc + n0 + col;
                *c = read_c ? scale_add(alpha, acc[i][j][r], beta, *c) : alpha * acc[i][j][r];
            }
        }
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
    __attribute__((amdgpu_waves_per_eu(WGM * WGN / 4))) gemm_pipe_kernel(GemmArgs p) {
    typedef PipeShape<T, BM, BN, BK, WGM, WGN> S;
    __shared__ u32x4_t lds[3 * S::STAGE];
    const int tiles_m = (int)((p.m + BM - 1) / BM);
    const int tiles_n = (int)((p.n + BN - 1) / BN);
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    pipe_tile<T, BM, BN, BK, WGM, WGN>(p, lds, tm, tn);
}

// Split-k with the three-stage tile: work-group (x, y) computes C tile x over
// the y-th range of kc values of k (a multiple of BK, so A and B keep their
// 16-byte alignment) with alpha = 1 and beta = 0 into plane y of W (m x n, row
// stride n); splitk_reduce_kernel sums the planes.
template <typename T, int BM, int BN, int BK, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
    __attribute__((amdgpu_waves_per_eu(WGM * WGN / 4)))
    gemm_pipe_splitk_kernel(GemmArgs p, int64_t kc, T *W) {
    typedef PipeShape<T, BM, BN, BK, WGM, WGN> S;
    __shared__ u32x4_t lds[3 * S::STAGE];
    const int tiles_m = (int)((p.m + BM - 1) / BM);
    const int tiles_n = (int)((p.n + BN - 1) / BN);
    int tm, tn;
    tile_of_block(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t y = blockIdx.y, k0 = y * kc;
    GemmArgs q = p;
    q.k = p.k - k0 < kc ? p.k - k0 : kc;
    q.A = (const T *)p.A + k0;
    q.B = (const T *)p.B + k0 * p.ldb;
    q.alpha = 1.0;
    q.beta = 0.0;
    q.C = W + y * p.m * p.n;
    q.ldc = p.n;
    pipe_tile<T, BM, BN, BK, WGM, WGN>(q, lds, tm, tn);
}

// ---------------------------------------------------------------------------
// Launchers and registries.
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC,
          bool ALIGN>
hipError_t launch_splitk(const GemmArgs &a, int S, int64_t kc, void *W, hipStream_t s) {
    int64_t blocks = ((a.m + BM - 1) / BM) * ((a.n + BN - 1) / BN);
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff || S < 1 || S > 65535) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((gemm_splitk_kernel<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, ALIGN>),
                       dim3((unsigned)blocks, (unsigned)S), dim3(64 * WGM * WGN), 0, s, a, kc,
                       (T *)W);
    return hipGetLastError();
}

// Split-k with the three-stage 128 x 128 eight-wave tile (k-step 16 for FP64, 32
// for FP32): its requirements are those of launch_pipe (16-byte rows and bases,
// 32-bit panel offsets); false if they do not hold.
bool pipe_splitk_eligible(const GemmArgs &a, int32_t dtype) {
    const int64_t es = dtype == MGEMM_F32 ? 4 : 8;
    const int64_t EPU = 16 / es, BM = 128, BN = 128, BK = dtype == MGEMM_F32 ? 32 : 16;
    return a.k >= 1 && a.n >= EPU && a.n % EPU == 0 && a.lda % EPU == 0 && a.ldb % EPU == 0 &&
           ((uintptr_t)a.A % 16) == 0 && ((uintptr_t)a.B % 16) == 0 &&
           BM * a.lda * es < ((int64_t)1 << 31) && (BK * a.ldb + BN) * es < ((int64_t)1 << 31);
}

hipError_t launch_pipe_splitk(const GemmArgs &a, int32_t dtype, int S, int64_t kc, void *W,
                              hipStream_t s) {
    if (!pipe_splitk_eligible(a, dtype)) return hipErrorInvalidValue;
    const int64_t blocks = ((a.m + 127) / 128) * ((a.n + 127) / 128);
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff || S < 1 || S > 65535) return hipErrorInvalidConfiguration;
    if (dtype == MGEMM_F32)
        hipLaunchKernelGGL((gemm_pipe_splitk_kernel<float, 128, 128, 32, 4, 2>),
                           dim3((unsigned)blocks, (unsigned)S), dim3(512), 0, s, a, kc, (float *)W);
    else
        hipLaunchKernelGGL((gemm_pipe_splitk_kernel<double, 128, 128, 16, 4, 2>),
                           dim3((unsigned)blocks, (unsigned)S), dim3(512), 0, s, a, kc,
                           (double *)W);
    return hipGetLastError();
}

hipError_t splitk_reduce(int32_t dtype, const void *W, int S, const GemmArgs &a, hipStream_t s) {
    const int64_t gx = std::min<int64_t>((a.n + 255) / 256, 64);
    const int64_t gy = std::min<int64_t>(a.m, 65535);
    if (dtype == MGEMM_F32)
        hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3((unsigned)gx, (unsigned)gy), dim3(256),
                           0, s, (const float *)W, S, a.m, a.n, (float)a.alpha, (float)a.beta,
                           a.beta != 0.0 ? 1 : 0, (float *)a.C, a.ldc);
    else
        hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3((unsigned)gx, (unsigned)gy),
                           dim3(256), 0, s, (const double *)W, S, a.m, a.n, a.alpha, a.beta,
                           a.beta != 0.0 ? 1 : 0, (double *)a.C, a.ldc);
    return hipGetLastError();
}

template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC>
hipError_t launch_batched(const BatchProblem *probs, const uint64_t *tile_map,
                          const int64_t *list_off, int nlist, int nprob,
                          unsigned long long *counters, int grid, hipStream_t s) {
    hipLaunchKernelGGL((gemm_batched_kernel<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC>),
                       dim3((unsigned)grid), dim3(64 * WGM * WGN), 0, s, probs, tile_map, list_off,
                       nlist, nprob, counters);
    return hipGetLastError();
}

// Resident work-groups per compute unit of the batched kernel (occupancy query).
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int EPT, int DBUF, int OCC>
int batched_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, gemm_batched_kernel<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC>,
            64 * WGM * WGN, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// The pipelined kernel where its requirements hold, else the two-stage kernel of
// the same tile (FWGM x FWGN waves), which sums in the same order.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, int FWGM, int FWGN, int FEPT>
hipError_t launch_pipe(const GemmArgs &a, hipStream_t s) {
    // 16-byte rows of A and B; 32-bit per-lane byte offsets: BM rows of A and BK
    // rows of B must span < 2^31 bytes
    constexpr int64_t EPU = 16 / (int64_t)sizeof(T);
    const bool ok = a.k >= 1 && a.n >= EPU && a.n % EPU == 0 && a.lda % EPU == 0 &&
                    a.ldb % EPU == 0 &&
                    ((uintptr_t)a.A % 16) == 0 && ((uintptr_t)a.B % 16) == 0 &&
                    (int64_t)BM * a.lda * (int64_t)sizeof(T) < ((int64_t)1 << 31) &&
                    ((int64_t)BK * a.ldb + BN) * (int64_t)sizeof(T) < ((int64_t)1 << 31);
    if (!ok) return launch_tiled<T, BM, BN, BK, FWGM, FWGN, FEPT, 1, 0, true>(a, s);
    int64_t blocks = ((a.m + BM - 1) / BM) * ((a.n + BN - 1) / BN);
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((gemm_pipe_kernel<T, BM, BN, BK, WGM, WGN>), dim3((unsigned)blocks),
                       dim3(64 * WGM * WGN), 0, s, a);
    return hipGetLastError();
}

// Registry entry of a pipelined configuration (double_buffer = 2: three stages);
// unaligned rows and batched plans use the two-stage kernel of the same tile.
// Its elems_per_thread is the elements of one 16-byte direct load; FWGM, FWGN and
// FEPT name the two-stage fallback (registered on its own as well).
#define MGEMM_PIPE_CFG(T, BM, BN, BK, WGM, WGN, FWGM, FWGN, FEPT)                      \
    {{BM, BN, BK, WGM * WGN, 16 / (int)sizeof(T), 2, WGM * WGN / 4},                      \
     &launch_pipe<T, BM, BN, BK, WGM, WGN, FWGM, FWGN, FEPT>,                             \
     &launch_tiled<T, BM, BN, BK, FWGM, FWGN, FEPT, 1, 0, false>,                         \
     &launch_batched<T, BM, BN, BK, FWGM, FWGN, FEPT, 1, 0>,                               \
     &batched_occupancy<T, BM, BN, BK, FWGM, FWGN, FEPT, 1, 0>}

// A two-stage configuration that also runs split-k for the built-in choice (FP64
// only: at N = 1024 it raised FP64 from 27.0 to 30.9 TFLOP/s, while FP32, twice as
// fast per tile, lost 4 % to the extra reduction).
#define MGEMM_REG_SPLITK(T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC)                       \
    {{BM, BN, BK, WGM * WGN, EPT, DBUF, OCC},                                             \
     &launch_tiled<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, true>,                        \
     &launch_tiled<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, false>,                       \
     &launch_batched<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC>,                             \
     &batched_occupancy<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC>,                          \
     {&launch_splitk<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, true>,                      \
      &launch_splitk<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, false>}}

#define MGEMM_CFG(T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC)                              \
    {{BM, BN, BK, WGM * WGN, EPT, DBUF, OCC},                                             \
     &launch_tiled<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, true>,                        \
     &launch_tiled<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC, false>,                       \
     &launch_batched<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC>,                             \
     &batched_occupancy<T, BM, BN, BK, WGM, WGN, EPT, DBUF, OCC>}

// (the 128 x 128 x 16 tile compiled for two waves per SIMD, one or two stages,
// spilled registers to scratch and is not registered)
static const KernelEntry kF64[] = {
    MGEMM_CFG(double, 128, 128, 16, 2, 2, 2, 1, 0),
    MGEMM_CFG(double, 128, 128, 32, 2, 2, 4, 1, 0),
    MGEMM_CFG(double, 256, 128, 16, 4, 2, 2, 1, 0),
    MGEMM_CFG(double, 128, 256, 16, 2, 4, 2, 1, 0),
    MGEMM_CFG(double, 128, 64, 16, 2, 2, 2, 1, 0),
    MGEMM_CFG(double, 128, 64, 32, 2, 2, 4, 0, 2),
    MGEMM_REG_SPLITK(double, 64, 64, 16, 2, 2, 2, 1, 0),
    MGEMM_CFG(double, 64, 64, 32, 2, 2, 2, 1, 0),
    MGEMM_REG_SPLITK(double, 32, 32, 16, 1, 1, 2, 1, 0),
    // three-stage direct-load kernels: the two large tiles with two waves per SIMD,
    // and a 64 x 64 tile with one (for products of a few hundred tiles: at 1024^3 it
    // ran at 47 TFLOP/s against 37 for the best two-stage tile; 64 x 64 x 16 reached
    // 40, 128 x 128 with four waves and 128 x 64 tiles 17-29)
    MGEMM_PIPE_CFG(double, 256, 128, 16, 4, 2, 4, 2, 2),
    MGEMM_PIPE_CFG(double, 128, 128, 16, 4, 2, 2, 2, 2),
    MGEMM_PIPE_CFG(double, 64, 64, 32, 2, 2, 2, 2, 4),
};

static const KernelEntry kF32[] = {
    MGEMM_CFG(float, 128, 128, 16, 2, 2, 2, 1, 0),
    MGEMM_CFG(float, 128, 128, 32, 2, 2, 4, 1, 0),
    MGEMM_CFG(float, 128, 128, 32, 2, 2, 4, 1, 2),
    MGEMM_CFG(float, 256, 128, 32, 4, 2, 4, 1, 0),
    MGEMM_CFG(float, 128, 256, 32, 2, 4, 4, 1, 0),
    MGEMM_CFG(float, 128, 64, 32, 2, 2, 4, 1, 0),
    MGEMM_CFG(float, 64, 64, 16, 2, 2, 2, 1, 0),
    MGEMM_CFG(float, 32, 32, 16, 1, 1, 2, 1, 0),
    MGEMM_PIPE_CFG(float, 256, 128, 32, 4, 2, 4, 2, 4),
    MGEMM_PIPE_CFG(float, 128, 128, 32, 4, 2, 2, 2, 4),
    // one wave per SIMD, 64 x 64 (1024^3: 89 TFLOP/s with k-steps of 64, 82 with 32,
    // against 62 for the best two-stage tile)
    MGEMM_PIPE_CFG(float, 64, 64, 64, 2, 2, 2, 2, 4),
    MGEMM_PIPE_CFG(float, 64, 64, 32, 2, 2, 2, 2, 4),
};

// The hand-registered entries followed by every part of the tuning grid.
static std::vector<KernelEntry> joined(const KernelEntry *hand, size_t nh,
                                       const GridPartFn *parts) {
    std::vector<KernelEntry> all(hand, hand + nh);
    for (int p = 0; p < GRID_PARTS; ++p) {
        int cnt = 0;
        const KernelEntry *e = parts[p](&cnt);
        all.insert(all.end(), e, e + cnt);
    }
    return all;
}

const KernelEntry *f64_registry(int *count) {
    static const std::vector<KernelEntry> all =
        joined(kF64, sizeof(kF64) / sizeof(kF64[0]), kGridF64Parts);
    *count = (int)all.size();
    return all.data();
}

const KernelEntry *f32_registry(int *count) {
    static const std::vector<KernelEntry> all =
        joined(kF32, sizeof(kF32) / sizeof(kF32[0]), kGridF32Parts);
    *count = (int)all.size();
    return all.data();
}

}  // namespace mgemm
