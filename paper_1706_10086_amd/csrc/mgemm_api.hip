// The C ABI of the library: argument checks, configuration choice and dispatch.
//
// Argument numbering and the -i convention follow the prototypes in mgemm.h:
// m=1 n=2 k=3 alpha=4 A=5 lda=6 B=7 ldb=8 beta=9 C=10 ldc=11 dtype=12 cfg=13
// stream=14.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include <algorithm>

#include "choice_table.h"
#include "mgemm_internal.h"

namespace mgemm {

static thread_local std::string g_err;
static hipStream_t g_stream = nullptr;

hipStream_t current_stream() { return g_stream; }

int32_t set_error(int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int32_t hip_error(hipError_t e, const char *where) {
    return set_error(MGEMM_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

size_t elem_size(int32_t dtype) {
    return dtype == MGEMM_F32 ? 4 : 8;
}

static bool ranges_overlap(const void *p, size_t pbytes, const void *q, size_t qbytes) {
    uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + qbytes && b < a + pbytes;
}

// Bytes spanned by an r x c row-major matrix with leading dimension ld.
static size_t span_bytes(int64_t r, int64_t c, int64_t ld, size_t es) {
    if (r <= 0 || c <= 0) return 0;
    return (size_t)((r - 1) * ld + c) * es;
}

// Checks the arguments in position order; returns 0 or -i.
int32_t check_args(int64_t m, int64_t n, int64_t k, double alpha, const void *A, int64_t lda,
                   const void *B, int64_t ldb, const void *C, int64_t ldc, int32_t dtype) {
    if (m < 0) return set_error(-1, "m < 0");
    if (n < 0) return set_error(-2, "n < 0");
    if (k < 0) return set_error(-3, "k < 0");
    const bool reads_ab = m > 0 && n > 0 && k > 0 && alpha != 0.0;
    if (reads_ab && A == nullptr) return set_error(-5, "A is NULL");
    if (lda < (k > 1 ? k : 1)) return set_error(-6, "lda < max(1,k)");
    if (reads_ab && B == nullptr) return set_error(-7, "B is NULL");
    if (ldb < (n > 1 ? n : 1)) return set_error(-8, "ldb < max(1,n)");
    if (m > 0 && n > 0 && C == nullptr) return set_error(-10, "C is NULL");
    if (ldc < (n > 1 ? n : 1)) return set_error(-11, "ldc < max(1,n)");
    if (dtype < MGEMM_F64 || dtype > MGEMM_CRT_INT8) return set_error(-12, "unknown dtype %d", dtype);
    if (reads_ab) {
        const size_t es = elem_size(dtype);
        const size_t cb = span_bytes(m, n, ldc, es);
        if (ranges_overlap(C, cb, A, span_bytes(m, k, lda, es)) ||
            ranges_overlap(C, cb, B, span_bytes(k, n, ldb, es)))
            return set_error(-10, "C overlaps A or B");
    }
    return 0;
}

// C = beta*C (k == 0 or alpha == 0); beta == 0 writes zeros without reading C.
template <typename T>
__global__ void scale_c_kernel(T *C, int64_t m, int64_t n, int64_t ldc, T beta) {
    int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx / n, j = idx - i * n;
        T *c = C + i * ldc + j;
        *c = beta == T(0) ? T(0) : beta * *c;
    }
}

int32_t scale_c(int32_t dtype, int64_t m, int64_t n, double beta, void *C, int64_t ldc,
                       hipStream_t s) {
    if (beta == 1.0) return 0;
    int64_t total = m * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dtype == MGEMM_F32)
        hipLaunchKernelGGL(scale_c_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (float *)C, m, n, ldc, (float)beta);
    else
        hipLaunchKernelGGL(scale_c_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (double *)C, m, n, ldc, beta);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : hip_error(e, "scale_c launch");
}

static const KernelEntry *registry(int32_t dtype, int *count) {
    switch (dtype) {
    case MGEMM_F64: return f64_registry(count);
    case MGEMM_F32: return f32_registry(count);
    default: *count = 0; return nullptr;
    }
}

static bool same_cfg(const mgemm_cfg &a, const mgemm_cfg &b) {
    return a.bm == b.bm && a.bn == b.bn && a.bk == b.bk && a.waves == b.waves &&
           a.elems_per_thread == b.elems_per_thread && a.double_buffer == b.double_buffer &&
           a.occupancy == b.occupancy;
}

// Built-in choice when no configuration is given: the first configuration of a
// preference list (largest tiles first, from square-size sweeps on MI355X) that
// still launches at least `min_tiles` work-groups; the last entry takes the rest.
struct Pref {
    mgemm_cfg cfg;
    int64_t min_tiles;
};

static const Pref kPrefF64[] = {
    {{256, 128, 16, 8, 2, 2, 2}, 512},
    {{128, 128, 16, 8, 2, 2, 2}, 256},
    {{128, 64, 32, 4, 4, 0, 2}, 256},
    {{64, 64, 16, 4, 2, 1, 0}, 256},
    {{32, 32, 16, 1, 2, 1, 0}, 0},
};

static const Pref kPrefF32[] = {
    {{256, 128, 32, 8, 4, 2, 2}, 512},
    {{128, 128, 32, 8, 4, 2, 2}, 256},
    {{128, 64, 32, 4, 4, 1, 0}, 256},
    {{64, 64, 16, 4, 2, 1, 0}, 256},
    {{32, 32, 16, 1, 2, 1, 0}, 0},
};

static const KernelEntry *find_entry(const KernelEntry *reg, int cnt, const mgemm_cfg &c);

static const KernelEntry *default_entry(int32_t dtype, const KernelEntry *reg, int cnt,
                                        int64_t m, int64_t n) {
    const Pref *pl = dtype == MGEMM_F32 ? kPrefF32 : kPrefF64;
    const int np = dtype == MGEMM_F32 ? (int)(sizeof kPrefF32 / sizeof kPrefF32[0])
                                      : (int)(sizeof kPrefF64 / sizeof kPrefF64[0]);
    for (int i = 0; i < np; ++i) {
        if (i + 1 < np && tiles_of(m, n, pl[i].cfg) < pl[i].min_tiles) continue;
        const KernelEntry *e = find_entry(reg, cnt, pl[i].cfg);
        if (e) return e;
    }
    return cnt > 0 ? &reg[0] : nullptr;
}

static const KernelEntry *find_entry(const KernelEntry *reg, int cnt, const mgemm_cfg &c) {
    for (int i = 0; i < cnt; ++i)
        if (same_cfg(reg[i].cfg, c)) return &reg[i];
    return nullptr;
}

// The configuration measured fastest for an m x n x k product whose rows are
// (rows16) or are not whole 16-byte loads (choice_table.h: the tuner database's
// shapes of the same class and log2 cell); NULL outside the table's range or for
// an unlisted cell.
// Whether m, n, k lie in the range the tuner's shapes cover ([64, 16384]).
static bool in_measured_range(int64_t m, int64_t n, int64_t k) {
    constexpr int64_t lo = (int64_t)1 << CHOICE_LOG2_LO, hi = (int64_t)1 << CHOICE_LOG2_HI;
    return m >= lo && n >= lo && k >= lo && m <= hi && n <= hi && k <= hi;
}

static const KernelEntry *measured_entry(int32_t dtype, bool rows16, int64_t m, int64_t n,
                                         int64_t k) {
    if (!in_measured_range(m, n, k)) return nullptr;
    auto lg = [](int64_t x) { int l = 0; while (x >> (l + 1)) ++l; return l; };
    const ChoiceCell key = {(int8_t)dtype, (int8_t)(rows16 ? 1 : 0), (int8_t)lg(m),
                            (int8_t)lg(n), (int8_t)lg(k)};
    auto less = [](const ChoiceCell &a, const ChoiceCell &b) {
        if (a.dtype != b.dtype) return a.dtype < b.dtype;
        if (a.rows16 != b.rows16) return a.rows16 < b.rows16;
        if (a.lm != b.lm) return a.lm < b.lm;
        if (a.ln != b.ln) return a.ln < b.ln;
        return a.lk < b.lk;
    };
    const ChoiceCell *end = kChoiceCells + CHOICE_CELLS;
    const ChoiceCell *c = std::lower_bound(kChoiceCells, end, key, less);
    if (c == end || less(key, *c)) return nullptr;
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    const mgemm_cfg cfg = {c->bm, c->bn, c->bk, c->waves, c->ept, c->dbuf, c->occ};
    return find_entry(reg, cnt, cfg);
}

// Whether the three-stage kernels can load these rows (16-byte rows and bases).
static bool rows_whole_loads(const GemmArgs &a, int32_t dtype) {
    const int64_t epu = dtype == MGEMM_F32 ? 4 : 2;
    return a.n % epu == 0 && a.lda % epu == 0 && a.ldb % epu == 0 &&
           ((uintptr_t)a.A % 16) == 0 && ((uintptr_t)a.B % 16) == 0;
}

static bool aligned_rows(const void *p, int64_t ld, size_t es) {
    return ((uintptr_t)p % (2 * es)) == 0 && (ld % 2) == 0;
}

// Whether A and B rows start on 2-element boundaries (the vector-load kernels).
bool rows_aligned(const void *A, int64_t lda, const void *B, int64_t ldb, int32_t dtype) {
    const size_t es = elem_size(dtype);
    return aligned_rows(A, lda, es) && aligned_rows(B, ldb, es);
}

// The registered kernel for (dtype, cfg), or the built-in choice for an m x n
// output when cfg is NULL.  On failure returns NULL with *err set (-13: cfg not
// registered; MGEMM_ERR_NOCONFIG: nothing registered).
const KernelEntry *choose_entry(int32_t dtype, int64_t m, int64_t n, const mgemm_cfg *cfg,
                                int32_t *err) {
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    *err = 0;
    if (cfg) {
        const KernelEntry *e = find_entry(reg, cnt, *cfg);
        if (!e)
            *err = set_error(-13, "configuration %dx%dx%d w%d e%d d%d o%d is not registered",
                             cfg->bm, cfg->bn, cfg->bk, cfg->waves, cfg->elems_per_thread,
                             cfg->double_buffer, cfg->occupancy);
        return e;
    }
    const KernelEntry *e = default_entry(dtype, reg, cnt, m, n);
    if (!e) *err = set_error(MGEMM_ERR_NOCONFIG, "no configuration for dtype %d", dtype);
    return e;
}

int32_t split_gemm(const GemmArgs &a, int32_t dtype, hipStream_t s);
int32_t model_choose(int32_t dtype, int64_t m, int64_t n, int64_t k, bool rows16, bool may_launch,
                     mgemm_cfg *out);

// Whether cfg is in dtype's registry.
bool cfg_registered(int32_t dtype, const mgemm_cfg &c) {
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    return reg && find_entry(reg, cnt, c) != nullptr;
}

// Whether work enqueued on s is being captured into a graph (then nothing may be
// launched and waited for on another stream); unknown counts as capturing.
static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return true;
    }
    return st != hipStreamCaptureStatusNone;
}

// Split-k for the built-in choice, before the measured choice for k >= 2048 and for
// shapes outside the measured range (m, n or k outside [64, 16384]); below that k
// the measured configurations, run whole, were faster (on 200 held-out FP64 shapes:
// split first for k >= 2048 only 0.990 of the better of the two per shape, split
// first always 0.932, never 0.917): when the preferred tile is a 64 x 64 or 32 x 32
// one and still leaves fewer than about four work-groups per compute unit, k is
// cut into S ranges of kc values (a multiple of SPLITK_MIN_K, itself a multiple of
// every tile's BK; the last range is the short one); the S partial products go to
// the library workspace and one reduction kernel adds them in order and applies
// alpha and beta.  The ranges run on the three-stage 128 x 128 tile (one
// work-group per compute unit; FP64 and FP32) when that fills at least three
// quarters of the compute units in one round, else, for FP64 only, on the chosen
// two-stage tile with about four work-groups per compute unit (for FP32, twice as
// fast per tile, that lost 4 % to the extra reduction, so FP32 then runs whole).
constexpr int64_t SPLITK_MIN_K = 256;
constexpr int64_t SPLITK_FIRST_K = 2048;
constexpr int SPLITK_MAX = 16;

static int compute_units() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = cus;
    }
    return cached[dev];
}

// S ranges wanted -> the ranges actually cut (kc rounded up to SPLITK_MIN_K)
static void cut_k(int64_t k, int64_t want, SplitPlan &sp) {
    want = std::min<int64_t>(std::min<int64_t>(want, k / SPLITK_MIN_K), SPLITK_MAX);
    if (want < 2) return;
    const int64_t kc = ((k + want - 1) / want + SPLITK_MIN_K - 1) / SPLITK_MIN_K * SPLITK_MIN_K;
    const int64_t S = (k + kc - 1) / kc;
    if (S < 2) return;
    sp.S = (int)S;
    sp.kc = kc;
}

static SplitPlan splitk_plan(const GemmArgs &a, const KernelEntry *e, int32_t dtype) {
    SplitPlan sp;
    const int cus = compute_units();
    const int64_t tiles = tiles_of(a.m, a.n, e->cfg);
    // only when the built-in choice fell back to a small tile for want of tiles
    if (cus <= 0 || tiles <= 0 || e->cfg.bm * e->cfg.bn > 64 * 64) return sp;
    if ((4 * (int64_t)cus + tiles - 1) / tiles < 2) return sp;       // enough tiles already
    if (pipe_splitk_eligible(a, dtype)) {
        const int64_t t128 = ((a.m + 127) / 128) * ((a.n + 127) / 128);
        SplitPlan pp;
        cut_k(a.k, cus / t128, pp);
        if (pp.S > 1 && 4 * t128 * pp.S >= 3 * (int64_t)cus) {
            pp.pipe = true;
            return pp;
        }
    }
    if (!e->splitk[0]) return sp;          // no two-stage split-k for this entry (FP32)
    cut_k(a.k, (4 * (int64_t)cus + tiles - 1) / tiles, sp);
    return sp;
}

// The partial products and their reduction, in W (the caller's buffer of at least
// S*m*n elements).
int32_t launch_splitk_into(const KernelEntry *e, const GemmArgs &a, int32_t dtype,
                                  bool al, const SplitPlan &sp, uint8_t *W, hipStream_t s) {
    hipError_t he = sp.pipe ? launch_pipe_splitk(a, dtype, sp.S, sp.kc, W, s)
                            : e->splitk[al ? 0 : 1](a, sp.S, sp.kc, W, s);
    if (he == hipSuccess) he = splitk_reduce(dtype, W, sp.S, a, s);
    return he == hipSuccess ? 0 : hip_error(he, "split-k launch");
}

// Split-k with its planes in the library workspace (grown on demand).
static int32_t run_splitk(const KernelEntry *e, const GemmArgs &a, int32_t dtype, bool al,
                          const SplitPlan &sp, hipStream_t s) {
    const size_t es = dtype == MGEMM_F32 ? 4 : 8;
    return with_workspace((size_t)sp.S * a.m * a.n * es, s, [&](uint8_t *W) -> int32_t {
        return launch_splitk_into(e, a, dtype, al, sp, W, s);
    });
}

// Three-stage tiles for rows that are whole 16-byte loads, each with the rate it
// sustains while every compute unit is busy (TFLOP/s: square N = 12288 on MI355X,
// calls back to back).  A product of T tiles of one of them runs in
// R = ceil(T / CUs) rounds that are T / (R CUs) full; the built-in choice takes
// the tile with the highest rate times fill when that fill is at least
// WAVE_FILL_MIN (fewer tiles than that: the measured table decides).  On the
// tuner's shapes with such rows this came 1.1 % (FP64) and 1.4-2.3 % (FP32) closer
// to the exhaustive best than the preference list and table alone; at N = 6144 FP64
// it takes the 128 x 128 tile (2304 tiles, 9 full rounds: 70 TFLOP/s) over the
// 256 x 128 one (1152 tiles, 4.5 rounds: 65).
struct PipeRate {
    mgemm_cfg cfg;
    double tflops;
};
static const PipeRate kPipeRatesF64[] = {{{256, 128, 16, 8, 2, 2, 2}, 72.5},
                                         {{128, 128, 16, 8, 2, 2, 2}, 70.4},
                                         {{64, 64, 32, 4, 2, 2, 1}, 54.2}};
static const PipeRate kPipeRatesF32[] = {{{256, 128, 32, 8, 4, 2, 2}, 141.0},
                                         {{128, 128, 32, 8, 4, 2, 2}, 135.1},
                                         {{64, 64, 32, 4, 4, 2, 1}, 120.6}};
constexpr double WAVE_FILL_MIN = 0.8;

// best_tf: the highest rate x fill among the tiles (0 without a device).
static const KernelEntry *wave_filled_pipe(const GemmArgs &a, int32_t dtype, double *best_tf,
                                           bool *best_large) {
    *best_tf = 0.0;
    *best_large = false;
    const int cus = compute_units();
    if (cus <= 0) return nullptr;
    const PipeRate *pr = dtype == MGEMM_F32 ? kPipeRatesF32 : kPipeRatesF64;
    constexpr int NP = 3;
    int best = -1;
    double score = 0.0, fill_best = 0.0;
    for (int i = 0; i < NP; ++i) {
        const int64_t t = tiles_of(a.m, a.n, pr[i].cfg);
        if (t <= 0) continue;
        const int64_t rounds = (t + cus - 1) / cus;
        const double fill = (double)t / (double)(rounds * cus);
        if (pr[i].tflops * fill > score) {
            score = pr[i].tflops * fill;
            fill_best = fill;
            best = i;
        }
    }
    *best_tf = score;
    *best_large = best >= 0 && pr[best].cfg.bm * pr[best].cfg.bn >= 128 * 128;
    if (best < 0 || fill_best < WAVE_FILL_MIN) return nullptr;
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    return find_entry(reg, cnt, pr[best].cfg);
}

// A split tail: where whole rounds of 128 x 128 tiles leave a last round of few
// tiles, the tile rows that fill whole rounds run whole and the remaining rows run
// with k cut into S ranges (S x their tiles <= CUs), so that the last round takes
// about 1/S of a round plus the sum of the S partial planes.  Taken when the
// estimate -- the main part at the tile's rate x its fill, the tail at
// TAIL_RATE_FACTOR of that rate x its fill (shorter k-loops), the sum at
// SUM_BYTES_PER_S -- beats plain_tf, the best single-tile estimate, by TAIL_GAIN,
// or by TAIL_GAIN_LARGE where that tile is a 128 x 128 or 256 x 128 one.
// (N = 3072 FP64: 21 of 24 tile rows whole in two full rounds, 3 rows in 3 ranges
// of 1024: 53 -> 65 TFLOP/s.  On the tuner's shapes whose estimate beat the best
// single tile by 2-5 %, the tail measured 1.003-1.073x as fast where that tile was
// 128 x 128 or 256 x 128, but 0.93-1.07x where it was 64 x 64.)
constexpr double TAIL_RATE_FACTOR = 0.8;
constexpr double SUM_BYTES_PER_S = 4e12;
constexpr double TAIL_GAIN = 1.05;
constexpr double TAIL_GAIN_LARGE = 1.02;

static bool split_tail_plan(const GemmArgs &a, int32_t dtype, double plain_tf, bool plain_large,
                            CallPlan &cp) {
    const int cus = compute_units();
    if (cus <= 0 || !pipe_splitk_eligible(a, dtype)) return false;
    const PipeRate &p = (dtype == MGEMM_F32 ? kPipeRatesF32 : kPipeRatesF64)[1];   // 128 x 128
    const int64_t tm = (a.m + 127) / 128, tn = (a.n + 127) / 128;
    const int64_t full = tm * tn / cus;                  // whole rounds
    if (full < 1) return false;
    const int64_t r1 = full * cus / tn;                  // tile rows run whole
    if (r1 < 1 || r1 >= tm) return false;
    const int64_t t1 = r1 * tn, t2 = (tm - r1) * tn;
    SplitPlan sp;
    cut_k(a.k, cus / t2, sp);
    if (sp.S < 2) return false;
    const int64_t main_rows = r1 * 128;
    const double w = 2.0 * (double)a.m * (double)a.n * (double)a.k * 1e-12;   // TFLOP
    const double wm = w * (double)main_rows / (double)a.m;
    const double fill_m = (double)t1 / (double)(((t1 + cus - 1) / cus) * cus);
    const double fill_t = std::min(1.0, (double)(t2 * sp.S) / (double)cus);
    const double sum_s = (double)(sp.S + 2) * (double)(a.m - main_rows) * (double)a.n *
                         (double)elem_size(dtype) / SUM_BYTES_PER_S;
    const double t = wm / (p.tflops * fill_m) + (w - wm) / (p.tflops * TAIL_RATE_FACTOR * fill_t) +
                     sum_s;
    if (w / t < (plain_large ? TAIL_GAIN_LARGE : TAIL_GAIN) * plain_tf) return false;
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    const KernelEntry *e = find_entry(reg, cnt, p.cfg);
    if (!e) return false;
    sp.pipe = true;
    cp.e = e;
    cp.sp = sp;
    cp.main_rows = main_rows;
    return true;
}

// What gemm_ex runs for one FP64 or FP32 product (CallPlan, mgemm_internal.h).
// A loaded cost model is evaluated on the device only when model_may_launch
// (else only its cached choices are used).
int32_t plan_call(const GemmArgs &a, int32_t dtype, const mgemm_cfg *cfg,
                         bool model_may_launch, CallPlan &cp) {
    int32_t err = 0;
    const KernelEntry *e = choose_entry(dtype, a.m, a.n, cfg, &err);
    if (!e) return err;
    cp.al = rows_aligned(a.A, a.lda, a.B, a.ldb, dtype);
    const bool in_range = in_measured_range(a.m, a.n, a.k);
    if (!cfg && (!in_range || a.k >= SPLITK_FIRST_K)) {
        // the preferred tile with k cut into ranges where that tile leaves the GPU
        // short of work: outside the range the tuner measured (and the model
        // learned), and inside it for long k
        cp.sp = splitk_plan(a, e, dtype);
    }
    if (!cfg && cp.sp.S == 1) {
        const bool rows16 = rows_whole_loads(a, dtype);
        if (in_range) {
            // a loaded cost model's choice (evaluated on the device once per shape)
            mgemm_cfg mc;
            const KernelEntry *me = nullptr;
            if (model_choose(dtype, a.m, a.n, a.k, rows16, model_may_launch, &mc) == 0) {
                int cnt = 0;
                const KernelEntry *reg = registry(dtype, &cnt);
                me = find_entry(reg, cnt, mc);
            }
            g_err.clear();     // a model that could not be used leaves the built-in choice
            if (me) {
                cp.e = me;
                return 0;
            }
        }
        // rows the three-stage kernels load: a split tail where it pays, else the
        // three-stage tile that fills the compute units' rounds best, where one
        // fills them well enough
        if (rows16) {
            double best_tf = 0.0;
            bool best_large = false;
            const KernelEntry *q = wave_filled_pipe(a, dtype, &best_tf, &best_large);
            if (split_tail_plan(a, dtype, best_tf, best_large, cp)) return 0;
            if (q) {
                cp.e = q;
                return 0;
            }
        }
        // the configuration measured fastest for shapes like this one: always for
        // rows the three-stage kernels cannot load (which the preference list
        // favours), else where the list names a two-stage configuration
        if (in_range && (!rows16 || e->cfg.double_buffer != 2)) {
            const KernelEntry *t = measured_entry(dtype, rows16, a.m, a.n, a.k);
            if (t) e = t;
        }
    }
    cp.e = e;
    return 0;
}

// gemm_ex: argument checks, configuration choice and launch.
static int32_t gemm_impl(int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                         int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                         int64_t ldc, int32_t dtype, const mgemm_cfg *cfg, void *stream) {
    g_err.clear();
    int32_t rc = check_args(m, n, k, alpha, A, lda, B, ldb, C, ldc, dtype);
    if (rc) return rc;
    // whether a call is valid does not depend on the values of alpha or beta
    if (dtype >= MGEMM_SPLIT_BF16 && cfg)
        return set_error(-13, "split dtypes take no tile configuration");
    hipStream_t s = stream ? (hipStream_t)stream : g_stream;
    if (m == 0 || n == 0) return 0;
    if (k == 0 || alpha == 0.0) {
        return scale_c(dtype == MGEMM_F32 ? MGEMM_F32 : MGEMM_F64, m, n, beta, C, ldc, s);
    }
    GemmArgs a{m, n, k, alpha, beta, A, lda, B, ldb, C, ldc};
    if (dtype >= MGEMM_SPLIT_BF16) return split_gemm(a, dtype, s);
    // calls on a capturing stream use cached model choices only
    CallPlan cp;
    rc = plan_call(a, dtype, cfg, !capturing(s) && !capturing(g_stream), cp);
    if (rc) return rc;
    if (cp.main_rows > 0) {
        GemmArgs am = a;
        am.m = cp.main_rows;
        hipError_t he = (cp.al ? cp.e->launch : cp.e->launch_unaligned)(am, s);
        if (he != hipSuccess) return hip_error(he, "gemm launch");
        return run_splitk(cp.e, rows_from(a, cp.main_rows, elem_size(dtype)), dtype, cp.al, cp.sp,
                          s);
    }
    if (cp.sp.S > 1) return run_splitk(cp.e, a, dtype, cp.al, cp.sp, s);
    hipError_t he = (cp.al ? cp.e->launch : cp.e->launch_unaligned)(a, s);
    if (he != hipSuccess) return hip_error(he, "gemm launch");
    return 0;
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int32_t gemm_ex(int64_t m, int64_t n, int64_t k, double alpha, const void *A, int64_t lda,
                const void *B, int64_t ldb, double beta, void *C, int64_t ldc, int32_t dtype,
                const mgemm_cfg *cfg, void *stream) {
    return gemm_impl(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, cfg, stream);
}

int32_t gemm(int64_t m, int64_t n, int64_t k, double alpha, const void *A, int64_t lda,
             const void *B, int64_t ldb, double beta, void *C, int64_t ldc, int32_t dtype) {
    return gemm_ex(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, nullptr, nullptr);
}

int32_t mgemm_set_stream(void *stream) {
    g_stream = (hipStream_t)stream;
    return 0;
}

const char *mgemm_last_error(void) { return g_err.c_str(); }

int32_t mgemm_config_count(int32_t dtype) {
    if (dtype < MGEMM_F64 || dtype > MGEMM_CRT_INT8) return -1;
    int cnt = 0;
    registry(dtype, &cnt);
    return cnt;
}

int32_t mgemm_host_alloc(int64_t bytes, int32_t coherent, void **host, void **dev) {
    if (!host || !dev) return set_error(-2, "host or dev is NULL");
    *host = *dev = nullptr;
    if (bytes <= 0) return set_error(-1, "bytes <= 0");
    const unsigned flags =
        hipHostMallocMapped | (coherent ? hipHostMallocCoherent : hipHostMallocNonCoherent);
    void *h = nullptr;
    hipError_t e = hipHostMalloc(&h, (size_t)bytes, flags);
    if (e != hipSuccess) return hip_error(e, "host_alloc: hipHostMalloc");
    void *d = nullptr;
    e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess || !d) {
        (void)hipHostFree(h);
        return hip_error(e != hipSuccess ? e : hipErrorInvalidValue,
                        "host_alloc: hipHostGetDevicePointer");
    }
    *host = h;
    *dev = d;
    return 0;
}

int32_t mgemm_host_free(void *host) {
    if (!host) return 0;
    hipError_t e = hipHostFree(host);
    return e == hipSuccess ? 0 : hip_error(e, "host_free: hipHostFree");
}

int32_t mgemm_config_flags(int32_t dtype, int32_t i) {
    if (dtype < MGEMM_F64 || dtype > MGEMM_CRT_INT8) return -1;
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    if (i < 0 || i >= cnt) return -2;
    const KernelEntry &e = reg[i];
    int32_t f = MGEMM_CFG_GEMM;
    if (e.batched) f |= MGEMM_CFG_BATCHED;
    if (e.splitk[0] || e.splitk[1]) f |= MGEMM_CFG_SPLITK;
    return f;
}

int32_t mgemm_choice(int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int32_t dtype,
                     mgemm_cfg *out, int32_t *splits, int64_t *main_rows) {
    g_err.clear();
    if (m < 1) return set_error(-1, "m < 1");
    if (n < 1) return set_error(-2, "n < 1");
    if (k < 1) return set_error(-3, "k < 1");
    if (lda < k) return set_error(-4, "lda < k");
    if (ldb < n) return set_error(-5, "ldb < n");
    if (dtype != MGEMM_F64 && dtype != MGEMM_F32)
        return set_error(-6, "dtype must be MGEMM_F64 or MGEMM_F32");
    if (!out) return set_error(-7, "out is NULL");
    if (!splits) return set_error(-8, "splits is NULL");
    // stand-in operands: 16-byte aligned addresses that are never dereferenced
    void *const base = (void *)(uintptr_t)256;
    GemmArgs a{m, n, k, 1.0, 0.0, base, lda, base, ldb, base, n};
    CallPlan cp;
    const int32_t rc = plan_call(a, dtype, nullptr, false, cp);
    if (rc) return rc;
    *splits = cp.sp.S;
    *out = cp.e->cfg;
    if (main_rows) *main_rows = cp.main_rows > 0 ? cp.main_rows : (cp.sp.S > 1 ? 0 : m);
    if (cp.sp.S > 1 && cp.sp.pipe) {
        // the three-stage 128 x 128 tile runs the ranges
        int cnt = 0;
        const KernelEntry *reg = registry(dtype, &cnt);
        for (int i = 0; i < cnt; ++i)
            if (reg[i].cfg.bm == 128 && reg[i].cfg.bn == 128 && reg[i].cfg.double_buffer == 2) {
                *out = reg[i].cfg;
                break;
            }
    }
    return 0;
}

int32_t mgemm_config_get(int32_t dtype, int32_t i, mgemm_cfg *out) {
    if (dtype < MGEMM_F64 || dtype > MGEMM_CRT_INT8) return -1;
    int cnt = 0;
    const KernelEntry *reg = registry(dtype, &cnt);
    if (i < 0 || i >= cnt) return -2;
    if (!out) return -3;
    *out = reg[i].cfg;
    return 0;
}

}  // extern "C"
