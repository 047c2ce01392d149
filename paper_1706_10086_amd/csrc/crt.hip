// Modular-integer emulation of an FP64 GEMM on int8 matrix cores (Ozaki scheme
// II: Ozaki, Uchino, Imamura, "Ozaki Scheme II: A GEMM-oriented emulation of
// floating-point matrix multiplication using an integer modular technique", 2025).
//
// C = alpha*A*B + beta*C with FP64 A, B, C:
//  1. scale     e_i, f_j: exponents of the row / column maxima (shared with the
//               slice emulation); b = the operand width, the largest b <= 62 with
//               k 2^(2b) <= 2^123.
//  2. residues  A'_ip = trunc(A_ip 2^(b - e_i)) and B'_pj = trunc(B_pj 2^(b - f_j))
//               are integers below 2^b; their residues modulo the 16 moduli below,
//               in [-p/2, p/2), are stored as int8 planes (B transposed, so both
//               operands are k-contiguous).
//  3. products  one int8 GEMM per modulus on the matrix cores with exact int32
//               accumulation (in launches of at most 2^16 k, each adding its
//               residues to the previous ones), whose result modulo p is stored as
//               one byte per element.
//  4. combine   the Chinese remainder theorem gives the exact integer
//               C'_ij = sum_p A'_ip B'_pj from its 16 residues (|C'| <= 2^123, a
//               quarter of the moduli's product), which is rounded once to FP64,
//               scaled by 2^(e_i + f_j - 2b) and the epilogue alpha*v + beta*C
//               applied.
//
// Against the slice emulation with int8 slices (36 slice-pair products of the
// same operand width), this needs 16 products of the full width, each a plain
// int8 GEMM.
#include <limits.h>

#include "mgemm_internal.h"

namespace mgemm {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Pairwise coprime moduli, the largest such set below 2^8: product > 2^125.37.

// The moduli as compile-time constants for the device (t is unrolled), so the
// residues use constant-divisor arithmetic.
__host__ __device__ constexpr int modulus(int t) {
    return t == 0 ? 256 : t == 1 ? 255 : t == 2 ? 253 : t == 3 ? 251 : t == 4 ? 247 :
           t == 5 ? 241 : t == 6 ? 239 : t == 7 ? 233 : t == 8 ? 229 : t == 9 ? 227 :
           t == 10 ? 223 : t == 11 ? 217 : t == 12 ? 211 : t == 13 ? 199 : t == 14 ? 197 : 193;
}
// 2^e mod p_t
__host__ __device__ constexpr int pow2_mod(int t, int e) {
    return (int)(((uint64_t)1 << e) % (uint64_t)modulus(t));
}
__constant__ int kModuliDev[CRT_MODULI] = {modulus(0),  modulus(1),  modulus(2),  modulus(3),
                                           modulus(4),  modulus(5),  modulus(6),  modulus(7),
                                           modulus(8),  modulus(9),  modulus(10), modulus(11),
                                           modulus(12), modulus(13), modulus(14), modulus(15)};

// ---------------------------------------------------------------------------
// 2. Residues.
// ---------------------------------------------------------------------------
// Residues of the integer a (|a| < 2^62, held exactly in a double) modulo each p,
// as int8 in [-p/2, p/2).  a = hi 2^32 + lo with 0 <= lo < 2^32, |hi| < 2^30, and in
// 16-bit digits a = h1 2^48 + h0 2^32 + l1 2^16 + l0 (h1 signed, |h1| < 2^14), so
// a = h1 c48 + h0 c32 + l1 c16 + l0 (mod p) with c_e = 2^e mod p < 2^8: a sum below
// 2^26 in magnitude of 24-bit products; a multiple of p above 2^22 makes it
// non-negative for one unsigned reduction.
__device__ inline void residues_of(double a, int8_t (&r)[CRT_MODULI]) {
    const double hi = floor(a * 0x1p-32);
    const double lo = a - hi * 0x1p32;
    const int hi_i = (int)hi;
    const uint32_t lo_u = (uint32_t)lo;
    const int h1 = hi_i >> 16, h0 = hi_i & 0xFFFF;
    const int l1 = (int)(lo_u >> 16), l0 = (int)(lo_u & 0xFFFFu);
#pragma unroll
    for (int t = 0; t < CRT_MODULI; ++t) {
        const int p = modulus(t);
        const int bias = p * ((1 << 22) / p + 1);              // > 2^22, multiple of p
        const int sum = __mul24(h1, pow2_mod(t, 48)) + __mul24(h0, pow2_mod(t, 32)) +
                        __mul24(l1, pow2_mod(t, 16)) + l0 + bias;
        int v = (int)((uint32_t)sum % (uint32_t)p);               // [0, p)
        if (v > (p - 1) / 2) v -= p;                              // [-p/2, p/2)
        r[t] = (int8_t)v;
    }
}

// Thread per (row, 8 consecutive k) of A; rows >= m and k >= k give zeros.
__global__ void __launch_bounds__(256)
crt_residue_a_kernel(const double *__restrict__ A, int64_t m, int64_t k, int64_t lda,
                     const int *__restrict__ e, int bits, int8_t *__restrict__ Q, int64_t mp,
                     int64_t kp) {
    const int64_t groups = kp / 8;
    const int64_t total = mp * groups;
    const int64_t plane = mp * kp;
    for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
         gid += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = gid / groups;
        const int64_t p0 = (gid - i * groups) * 8;
        const int ex = i < m ? e[i] : 0;
        uint32_t w[CRT_MODULI][2];
#pragma unroll
        for (int t = 0; t < CRT_MODULI; ++t) w[t][0] = w[t][1] = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t p = p0 + v;
            const double x = (i < m && p < k) ? trunc(ldexp(A[i * lda + p], bits - ex)) : 0.0;
            int8_t r[CRT_MODULI];
            residues_of(x, r);
#pragma unroll
            for (int t = 0; t < CRT_MODULI; ++t)
                w[t][v >> 2] |= (uint32_t)(uint8_t)r[t] << (8 * (v & 3));
        }
#pragma unroll
        for (int t = 0; t < CRT_MODULI; ++t)
            *(uint2 *)(Q + t * plane + i * kp + p0) = make_uint2(w[t][0], w[t][1]);
    }
}

// 64 (k) x 64 (n) tile of B through LDS; thread (column j, 16 consecutive k) ->
// the residues of column j, stored k-contiguous.
__global__ void __launch_bounds__(256)
crt_residue_b_kernel(const double *__restrict__ B, int64_t k, int64_t n, int64_t ldb,
                     const int *__restrict__ fexp, int bits, int8_t *__restrict__ Q, int64_t np,
                     int64_t kp) {
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
    uint32_t w[CRT_MODULI][4];
#pragma unroll
    for (int t = 0; t < CRT_MODULI; ++t) w[t][0] = w[t][1] = w[t][2] = w[t][3] = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const double x = trunc(ldexp(tile[pg + v][jc], bits - ex));
        int8_t r[CRT_MODULI];
        residues_of(x, r);
#pragma unroll
        for (int t = 0; t < CRT_MODULI; ++t)
            w[t][v >> 2] |= (uint32_t)(uint8_t)r[t] << (8 * (v & 3));
    }
    const int64_t plane = np * kp;
#pragma unroll
    for (int t = 0; t < CRT_MODULI; ++t)
        *(u32x4 *)(Q + t * plane + j * kp + p0 + pg) = u32x4{w[t][0], w[t][1], w[t][2], w[t][3]};
}

// ---------------------------------------------------------------------------
// 3. One int8 GEMM per modulus.
// ---------------------------------------------------------------------------
// Work-group: WGM x WGN waves own a 256 x 256 tile of C for one modulus; each
// wave a (256/WGM) x (256/WGN) block as 32x32 accumulators of the 32x32x32 int8
// MFMA.  A stage holds 64 k of the tile's 256 A rows and 256 B columns; the
// stages are filled by direct global->LDS loads NST-1 stages ahead, and every
// fragment register is refilled from the next stage right after its last use.
// Operands are zero-padded to whole tiles and stages, so no load or store needs
// a bounds test.
constexpr int G_KS = CRT_KSTEP;                 // k per stage
constexpr int G_PASS = (1 << 16) / G_KS;        // stages per launch: |acc| < 2^16 * 2^14

// LDS layout of one stage: 256 A rows then 256 B rows of 64 k (4 units of 16 B).
//  PADDED:   rows of 5 units (the fifth a copy, never read); four stages.
//  SWIZZLED: rows of 4 units, logical unit c of row r stored at c ^ sw(r) with
//            sw(r) = (r >> 2) & 3; five stages in the same space.
// Both keep the fragment reads free of bank conflicts (SQ_LDS_BANK_CONFLICT reads
// 0 for either; of the XOR patterns tried, (r >> 1) & 3 or ((r >> 1) ^ (r >> 3)) & 3
// conflict on half of the LDS cycles, r & 3 on three quarters).
template <bool SWZ> struct StageLayout {
    static constexpr int ROW = SWZ ? 4 : 5;                 // units per LDS row
    static constexpr int AUNITS = CRT_TILE * ROW;           // A part of a stage
    static constexpr int STAGE = 2 * AUNITS;                // units per stage
    static constexpr int NST = SWZ ? 5 : 4;                 // stages
    static_assert(AUNITS % 64 == 0, "a wave's loads lie in one operand");
    static_assert(NST * STAGE * 16 <= 163840, "LDS");
    __device__ static int sw(int r) { return SWZ ? (r >> 2) & 3 : 0; }
};

struct CrtGemmArgs {
    const int8_t *QA;
    const int8_t *QB;
    uint8_t *R;
    int64_t plane_a, plane_b, plane_r;
    int64_t kp, np;
    int tiles_m, tiles_n;
    int ch0, ch1;          // stages [ch0, ch1) of this pass (at most 2^16 k)
    int accumulate;        // add the previous passes' residues already in R
};

// 32x32 accumulator element r of lane l: row 8(r/4) + 4(l/32) + r%4, column l%32.
__device__ inline int crt_acc_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

template <int WGM, int WGN, bool SWZ>
__global__ void __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(WGM * WGN / 4)))
crt_gemm_kernel(CrtGemmArgs a) {
    typedef StageLayout<SWZ> L;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WTM = CRT_TILE / WGM, WTN = CRT_TILE / WGN;   // wave block
    constexpr int FM = WTM / 32, FN = WTN / 32;                 // accumulators per wave
    constexpr int LOADS = L::STAGE / NT;                        // loads per lane per stage
    constexpr int NST = L::NST;
    static_assert(L::STAGE % NT == 0, "load split");
    __shared__ u32x4 lds[NST * L::STAGE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WGN, wn = wave % WGN;

    // work-group -> (modulus, tile): the moduli one after another, each walked as
    // one GEMM's tiles (XCD-aware, grouped rows)
    const int tiles = a.tiles_m * a.tiles_n;
    int lid = blockIdx.x;
    {
        const int full = (int)(gridDim.x / 8) * 8;
        if (lid < full) lid = (lid % 8) * (full / 8) + lid / 8;
    }
    const int t = lid / tiles;
    int tm, tn;
    tile_of_block(lid - t * tiles, 0, a.tiles_m, a.tiles_n, tm, tn);
    const int p = kModuliDev[t];
    const int8_t *qa = a.QA + t * a.plane_a + (int64_t)tm * CRT_TILE * a.kp;
    const int8_t *qb = a.QB + t * a.plane_b + (int64_t)tn * CRT_TILE * a.kp;

    // per-lane source offsets: LDS unit u of a stage holds row r, logical unit c
    uint32_t off[LOADS];
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
        const int u = i * NT + wave * 64 + lane;
        const int v = u < L::AUNITS ? u : u - L::AUNITS;
        const int r = v / L::ROW, pu = v % L::ROW;
        const int c = SWZ ? (pu ^ L::sw(r)) : (pu < 4 ? pu : 3);
        off[i] = (uint32_t)r * (uint32_t)a.kp + (uint32_t)c * 16u;
    }
    // load instruction i of chunk `chunk` into stage st
    auto issue_one = [&](int i, int chunk, int st) {
        const int first = i * NT + wave * 64;                     // uniform per wave
        const int8_t *src = (first < L::AUNITS ? qa : qb) + (int64_t)chunk * G_KS + off[i];
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (__attribute__((address_space(3))) void *)(lds + st * L::STAGE + first),
                                         16, 0, 0);
    };
    auto issue = [&](int chunk, int st) {
#pragma unroll
        for (int i = 0; i < LOADS; ++i) issue_one(i, chunk, st);
    };

    v16i acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v16i{};

    // fragment rows of this lane: the swizzle is the same for rows 32 apart
    const int ra = wm * WTM + (lane & 31), rb = wn * WTN + (lane & 31);
    int a_unit[2], b_unit[2];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const int c = kk * 2 + (lane >> 5);
        a_unit[kk] = ra * L::ROW + (c ^ L::sw(ra));
        b_unit[kk] = L::AUNITS + rb * L::ROW + (c ^ L::sw(rb));
    }
    v4i fa[2][FM], fb[2][FN];
    auto read_a = [&](const u32x4 *st, int kk, int mt) {
        fa[kk][mt] = __builtin_bit_cast(v4i, st[a_unit[kk] + mt * 32 * L::ROW]);
    };
    auto read_b = [&](const u32x4 *st, int kk, int nt) {
        fb[kk][nt] = __builtin_bit_cast(v4i, st[b_unit[kk] + nt * 32 * L::ROW]);
    };
    // products of one stage; each fragment is refilled from the next stage right
    // after its last use (past the last stage the refills read a stale stage and
    // are never used)
    // The stage's loads (chunk lc into stage ls) are spread over the products, one
    // after every 2*FM/LOADS fragment rows, so that the memory pipeline takes them
    // a few at a time instead of all waves queueing every load at the barrier.
    auto products = [&](const u32x4 *nst, int lc, int ls) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int mt = 0; mt < FM; ++mt) {
#pragma unroll
                for (int nt = 0; nt < FN; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[kk][mt], fb[kk][nt],
                                                                         acc[mt][nt], 0, 0, 0);
                read_a(nst, kk, mt);
                constexpr int every = 2 * FM / LOADS > 0 ? 2 * FM / LOADS : 1;
                static_assert((LOADS - 1) * every < 2 * FM, "every load gets a slot");
                const int slot = kk * FM + mt;
                if (slot % every == 0 && slot / every < LOADS) issue_one(slot / every, lc, ls);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int nt = 0; nt < FN; ++nt) read_b(nst, kk, nt);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // stages of this pass, counted from its first.  Chunks 0..NST-2 in flight;
    // wait for chunk 0 (the loads of NST-2 chunks may remain)
    qa += (int64_t)a.ch0 * G_KS;
    qb += (int64_t)a.ch0 * G_KS;
    const int nst = a.ch1 - a.ch0;
#pragma unroll
    for (int c = 0; c < NST - 1; ++c) issue(c < nst ? c : nst - 1, c);
    __builtin_amdgcn_s_waitcnt(vmcnt_imm((NST - 2) * LOADS));
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
        for (int mt = 0; mt < FM; ++mt) read_a(lds, kk, mt);
#pragma unroll
        for (int nt = 0; nt < FN; ++nt) read_b(lds, kk, nt);
    }
    int st = 0;                                   // stage of chunk c
    for (int c = 0; c < nst; ++c) {
        // chunk c+1 has landed (the loads of NST-3 later chunks may remain)
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((NST - 3) * LOADS));
        __syncthreads();
        const int st1 = st + 1 == NST ? 0 : st + 1;
        const int stn = st == 0 ? NST - 1 : st - 1;    // stage of chunk c-1
        // chunk c+NST-1 into the stage of chunk c-1 (past the end: the last chunk
        // again, in bounds and never used)
        products(lds + st1 * L::STAGE, c + NST - 1 < nst ? c + NST - 1 : nst - 1, stn);
        st = st1;
    }
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));       // no load lands after this point

    uint8_t *R = a.R + t * a.plane_r;
    const int64_t row0 = (int64_t)tm * CRT_TILE + wm * WTM;
    const int64_t col0 = (int64_t)tn * CRT_TILE + wn * WTN + (lane & 31);
#pragma unroll
    for (int mt = 0; mt < FM; ++mt)
#pragma unroll
        for (int nt = 0; nt < FN; ++nt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                uint8_t *dst = R + (row0 + mt * 32 + crt_acc_row(lane, r)) * a.np + col0 + nt * 32;
                int v = acc[mt][nt][r] % p;
                if (a.accumulate) v += *dst;
                v %= p;
                if (v < 0) v += p;
                *dst = (uint8_t)v;
            }
}

// ---------------------------------------------------------------------------
// 4. Chinese-remainder reconstruction, one rounding, epilogue.
// ---------------------------------------------------------------------------
// With P the moduli's product, M_t = P / p_t and W_t = M_t (M_t^-1 mod p_t) < P,
// S = sum_t r_t W_t is congruent to C' modulo P; q = round(S / P) is found from
// sum_t r_t (W_t / P) in FP64 (|C'| <= P/4 keeps S/P within 1/4 of q, far above
// the estimate's error), and C' = S - q P is computed modulo 2^128, which is exact
// because |C'| < 2^127.
struct CrtReconArgs {
    uint32_t w[CRT_MODULI][4];      // W_t as four 32-bit limbs, least significant first
    double wf[CRT_MODULI];          // W_t / P
    uint32_t pl[4];                 // P as four 32-bit limbs
};

// Signed 128-bit integer (hi, lo) -> FP64, rounded to nearest even.
__device__ inline double i128_to_double(uint64_t hi, uint64_t lo) {
    const bool neg = (int64_t)hi < 0;
    if (neg) {
        lo = ~lo + 1;
        hi = ~hi + (lo == 0 ? 1 : 0);
    }
    double v;
    if (hi == 0) {
        v = (double)lo;                            // one rounding of an exact sum
    } else {
        const int lz = __clzll((long long)hi);     // 0..63
        const int drop = 64 - lz;                  // bits below the top 64
        const uint64_t top = lz == 0 ? hi : (hi << lz) | (lo >> drop);
        const uint64_t rest = lz == 0 ? lo : lo << lz;
        // a nonzero remainder below the top 64 bits turns an exact half into
        // "above half"; it cannot change any other rounding decision
        v = ldexp((double)(top | (rest != 0 ? 1 : 0)), drop);
    }
    return neg ? -v : v;
}

// C' of one element from its 16 residues r_t (byte v of each word rr[t]).
__device__ inline double crt_value(const uint64_t (&rr)[CRT_MODULI], int v, const CrtReconArgs &rc) {
    // S = sum_t r_t W_t by 32-bit limbs: each limb sum < 16 * 255 * 2^32 < 2^44
    // (measured faster than 20-bit limbs with 24-bit multiplies)
    uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    double qf = 0.0;
#pragma unroll
    for (int t = 0; t < CRT_MODULI; ++t) {
        const uint32_t r = (uint32_t)(rr[t] >> (8 * v)) & 0xFFu;
        s0 += (uint64_t)r * rc.w[t][0];
        s1 += (uint64_t)r * rc.w[t][1];
        s2 += (uint64_t)r * rc.w[t][2];
        s3 += (uint64_t)r * rc.w[t][3];
        qf = fma((double)r, rc.wf[t], qf);
    }
    const uint32_t q = (uint32_t)rint(qf);         // < 16 * 256
    // subtract q P limb by limb (q P_l < 2^44); carries propagate as signed values,
    // everything modulo 2^128
    int64_t d0 = (int64_t)s0 - (int64_t)((uint64_t)q * rc.pl[0]);
    int64_t d1 = (int64_t)s1 - (int64_t)((uint64_t)q * rc.pl[1]) + (d0 >> 32);
    int64_t d2 = (int64_t)s2 - (int64_t)((uint64_t)q * rc.pl[2]) + (d1 >> 32);
    int64_t d3 = (int64_t)s3 - (int64_t)((uint64_t)q * rc.pl[3]) + (d2 >> 32);
    const uint64_t lo = ((uint64_t)(uint32_t)d1 << 32) | (uint32_t)d0;
    const uint64_t hi = ((uint64_t)(uint32_t)d3 << 32) | (uint32_t)d2;
    return i128_to_double(hi, lo);
}

// Thread per 8 consecutive elements of a row of C: one 8-byte load per modulus.
__global__ void __launch_bounds__(256)
crt_reconstruct_kernel(const uint8_t *__restrict__ R, int64_t plane_r, int64_t np,
                       const int *__restrict__ e, const int *__restrict__ fexp, int two_bits,
                       double *__restrict__ C, int64_t m, int64_t n, int64_t ldc, double alpha,
                       double beta, CrtReconArgs rc) {
    const int64_t n8 = (n + 7) / 8;
    const int64_t total = m * n8;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / n8, j0 = (idx - i * n8) * 8;
        uint64_t rr[CRT_MODULI];
#pragma unroll
        for (int t = 0; t < CRT_MODULI; ++t)
            rr[t] = *(const uint64_t *)(R + t * plane_r + i * np + j0);
        const int ei = e[i];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t j = j0 + v;
            if (j >= n) break;
            const double cv = crt_value(rr, v, rc);
            const int fe = fexp[j];
            const double val = ldexp(cv, ei + (fe == INT_MIN ? 0 : fe) - two_bits);
            double *c = C + i * ldc + j;
            if (beta == 0.0) {
                *c = alpha * val;
            } else {
#pragma clang fp contract(off)
                *c = alpha * val + beta * *c;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
namespace {

struct CrtTables {
    CrtReconArgs rc;
    CrtTables() {
        typedef unsigned __int128 u128;
        u128 P = 1;
        for (int t = 0; t < CRT_MODULI; ++t) P *= (u128)modulus(t);
        for (int t = 0; t < CRT_MODULI; ++t) {
            const int p = modulus(t);
            const u128 M = P / (u128)p;
            // inverse of M mod p by the extended Euclidean algorithm
            long long r0 = (long long)(M % (u128)p), r1 = p, s0 = 1, s1 = 0;
            while (r1 != 0) {
                const long long qq = r0 / r1;
                long long tmp = r0 - qq * r1; r0 = r1; r1 = tmp;
                tmp = s0 - qq * s1; s0 = s1; s1 = tmp;
            }
            const long long inv = ((s0 % p) + p) % p;       // r0 == 1: coprime moduli
            const u128 W = M * (u128)inv;                    // < P: inv < p
            for (int l = 0; l < 4; ++l) rc.w[t][l] = (uint32_t)(W >> (32 * l));
            rc.wf[t] = (double)W / (double)P;
        }
        for (int l = 0; l < 4; ++l) rc.pl[l] = (uint32_t)(P >> (32 * l));
    }
};

const CrtTables &tables() {
    static const CrtTables tb;
    return tb;
}

}  // namespace

// The operand width b: the largest b <= 62 with k 2^(2b) <= 2^123, i.e.
// k <= 2^(123 - 2b) (at least 1).
int crt_operand_bits(int64_t k) {
    int b = 62;
    for (; b > 1; --b) {
        const int sh = 123 - 2 * b;
        if (sh >= 0 && (sh >= 63 || k <= ((int64_t)1 << sh))) break;
    }
    return b;
}

hipError_t crt_launch(const GemmArgs &g, hipStream_t s, const int *e, const int *fexp, int bits,
                      int8_t *QA, int8_t *QB, uint8_t *R, int64_t mp, int64_t np, int64_t kp) {
    const CrtTables &tb = tables();
    {
        const int64_t groups = mp * (kp / 8);
        int64_t blocks = (groups + 255) / 256;
        if (blocks > 1 << 20) blocks = 1 << 20;
        hipLaunchKernelGGL(crt_residue_a_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double *)g.A, g.m, g.k, g.lda, e, bits, QA, mp, kp);
        hipLaunchKernelGGL(crt_residue_b_kernel, dim3((unsigned)(np / 64), (unsigned)(kp / 64)),
                           dim3(256), 0, s, (const double *)g.B, g.k, g.n, g.ldb, fexp, bits, QB,
                           np, kp);
    }
    {
        CrtGemmArgs ga;
        ga.QA = QA;
        ga.QB = QB;
        ga.R = R;
        ga.plane_a = mp * kp;
        ga.plane_b = np * kp;
        ga.plane_r = mp * np;
        ga.kp = kp;
        ga.np = np;
        ga.tiles_m = (int)(mp / CRT_TILE);
        ga.tiles_n = (int)(np / CRT_TILE);
        const int64_t nstages = kp / CRT_KSTEP;
        const int64_t blocks = (int64_t)ga.tiles_m * ga.tiles_n * CRT_MODULI;
        // passes of at most 2^16 k keep the int32 sums exact; later passes add
        // their residues to the stored ones
        for (int64_t c0 = 0; c0 < nstages; c0 += G_PASS) {
            ga.ch0 = (int)c0;
            ga.ch1 = (int)(c0 + G_PASS < nstages ? c0 + G_PASS : nstages);
            ga.accumulate = c0 > 0;
            // 8 waves of 128 x 64 (two per SIMD) measured faster than 4 waves of
            // 128 x 128 (one per SIMD), which spend more time exposed at the barrier
            // (the swizzled five-stage layout measured 3 % faster than the padded
            // four-stage one)
            hipLaunchKernelGGL((crt_gemm_kernel<2, 4, true>), dim3((unsigned)blocks), dim3(512), 0, s, ga);
        }
    }
    {
        const int64_t total = g.m * ((g.n + 7) / 8);
        int64_t blocks = (total + 255) / 256;
        if (blocks > 1 << 20) blocks = 1 << 20;
        hipLaunchKernelGGL(crt_reconstruct_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const uint8_t *)R, mp * np, np, e, fexp, 2 * bits, (double *)g.C, g.m,
                           g.n, g.ldc, g.alpha, g.beta, tb.rc);
    }
    return hipGetLastError();
}

}  // namespace mgemm
