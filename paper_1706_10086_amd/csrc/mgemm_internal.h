// Internal declarations shared by the HIP kernel files and the C-ABI layer.
#pragma once

#include <functional>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mgemm.h"

namespace mgemm {

// Arguments of one GEMM, already validated on the host.
struct GemmArgs {
    int64_t m, n, k;
    double alpha, beta;
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
};

// One problem of a batched launch.  tile0 is the number of the problem's first
// C tile in the launch's work list; tiles_n the tile columns of the problem.
struct BatchProblem {
    GemmArgs g;
    int64_t tile0;
    int64_t tiles_n;
    int64_t aligned;    // 1: rows of A and B start on 2-element boundaries
};

// A registered kernel: its configuration and its launchers.  The batched kernel
// takes problems of any row alignment and picks each tile's load path from
// BatchProblem::aligned.
typedef hipError_t (*LaunchFn)(const GemmArgs &, hipStream_t);
typedef hipError_t (*BatchLaunchFn)(const BatchProblem *, const uint64_t *, const int64_t *, int,
                                    int, unsigned long long *, int, hipStream_t);

// Work lists of a batched launch: with a tile map, one list per XCD (work-group
// b starts on list b % BATCH_LISTS, the XCD it runs on, and then takes from the
// others); without one, a single list of tile numbers.  List l holds entries
// [off[l], off[l+1]) and has its own counter.
constexpr int BATCH_LISTS = 8;

// Tile map of a batched launch: entry t packs the problem index of tile t (bits
// 40-63) and the tile's row and column within that problem (bits 20-39, 0-19).
constexpr int TILE_MAP_PROB_BITS = 24, TILE_MAP_RC_BITS = 20;
inline uint64_t tile_map_entry(uint64_t prob, uint64_t tm, uint64_t tn) {
    return (prob << (2 * TILE_MAP_RC_BITS)) | (tm << TILE_MAP_RC_BITS) | tn;
}
typedef int (*OccupancyFn)();
// Split-k partial products: (GEMM, number of splits S, k per split, W): plane y of
// W (m x n, row stride n) receives the product over k range [y*kc, (y+1)*kc).
typedef hipError_t (*SplitkLaunchFn)(const GemmArgs &, int, int64_t, void *, hipStream_t);

struct KernelEntry {
    mgemm_cfg cfg;
    LaunchFn launch;             // aligned rows
    LaunchFn launch_unaligned;   // any rows
    BatchLaunchFn batched;               // any rows (per-problem load path)
    OccupancyFn batched_occupancy;
    SplitkLaunchFn splitk[2];            // split-k partials, [0] aligned rows, [1] any
                                         // rows; null where the tile has none
};

// A part of the tuning-grid registry (grid_*.hip, written by gen_grid.py).
typedef const KernelEntry *(*GridPartFn)(int *count);

// Per-dtype registries, defined in the kernel files: the hand-registered
// configurations, then the tuning-grid ones.
const KernelEntry *f64_registry(int *count);
const KernelEntry *f32_registry(int *count);

// ---------------------------------------------------------------------------
// Work-group id -> C tile.
// ---------------------------------------------------------------------------
// The hardware hands consecutive work-group ids to the 8 XCDs in turn.  First
// undo that dealing, so that logical ids [x*per, (x+1)*per) all run on XCD x;
// then walk tiles in groups of GROUP_M tile-rows, column by column, so that a
// run of consecutive logical ids covers a compact rectangle of C.
__device__ inline void tile_of_block(int bid, int nblocks, int tiles_m, int tiles_n,
                                     int &tm, int &tn) {
    constexpr int XCDS = 8;
    constexpr int GROUP_M = 8;
    int full = (nblocks / XCDS) * XCDS;
    int lid = bid;
    if (bid < full) {
        int per = full / XCDS;
        lid = (bid % XCDS) * per + bid / XCDS;
    }
    int group_size = GROUP_M * tiles_n;
    int group = lid / group_size;
    int first_m = group * GROUP_M;
    int gm = tiles_m - first_m < GROUP_M ? tiles_m - first_m : GROUP_M;
    int in_group = lid - group * group_size;
    tm = first_m + in_group % gm;
    tn = in_group / gm;
}

// Modular-integer (Ozaki scheme II) emulation: operands are padded to whole
// CRT_TILE x CRT_KSTEP blocks; crt_launch runs the residue, product and
// reconstruction kernels on exponents already computed (e per row of A, fexp per
// column of B, INT_MIN for an all-zero column).  Workspace: QA and QB hold
// CRT_MODULI int8 planes of mp x kp and np x kp, R CRT_MODULI byte planes of
// mp x np.
constexpr int CRT_MODULI = 16;
constexpr int CRT_TILE = 256;
constexpr int CRT_KSTEP = 64;
int crt_operand_bits(int64_t k);
hipError_t crt_launch(const GemmArgs &g, hipStream_t s, const int *e, const int *fexp, int bits,
                      int8_t *QA, int8_t *QB, uint8_t *R, int64_t mp, int64_t np, int64_t kp);

// Split-k partials with the three-stage 128 x 128 tile, FP64 or FP32 (dtype;
// otherwise the contract of SplitkLaunchFn); hipErrorInvalidValue unless
// pipe_splitk_eligible.
bool pipe_splitk_eligible(const GemmArgs &a, int32_t dtype);
hipError_t launch_pipe_splitk(const GemmArgs &a, int32_t dtype, int S, int64_t kc, void *W,
                              hipStream_t s);

// C = alpha * (sum of the S partial planes of W, in plane order) + beta * C.
hipError_t splitk_reduce(int32_t dtype, const void *W, int S, const GemmArgs &a, hipStream_t s);

// Runs fn on the current device's library-owned workspace grown to at least
// `bytes`, ordered on stream s after the workspace's previous user; returns fn's
// result (or an allocation error).
int32_t with_workspace(size_t bytes, hipStream_t s, const std::function<int32_t(uint8_t *)> &fn);

// The split of k of the built-in choice (split-k): S ranges of kc values each;
// S = 1 means no split.
struct SplitPlan {
    int S = 1;              // number of k ranges (1: no split)
    int64_t kc = 0;         // k per range
    bool pipe = false;      // three-stage 128 x 128 tile
};

// What gemm_ex runs for one FP64 or FP32 product: the kernel entry, whether A
// and B rows take vector loads (al), and for the built-in choice the split of k.
// With main_rows > 0, rows [0, main_rows) run whole on e and only the remaining
// rows run the split (a tail that would otherwise leave most compute units idle
// in a last round).
struct CallPlan {
    const KernelEntry *e = nullptr;
    bool al = false;
    SplitPlan sp;
    int64_t main_rows = 0;
};

// Rows [r, m) of a product: A and C start r rows further on.
inline GemmArgs rows_from(const GemmArgs &a, int64_t r, size_t es) {
    GemmArgs t = a;
    t.m = a.m - r;
    t.A = (const char *)a.A + (size_t)(r * a.lda) * es;
    t.C = (char *)a.C + (size_t)(r * a.ldc) * es;
    return t;
}

// gemm_ex's choice for a checked, non-trivial FP64/FP32 product (cfg: the
// caller's configuration or NULL); a loaded cost model is evaluated on the
// device only when model_may_launch, else only its cached choices count.
int32_t plan_call(const GemmArgs &a, int32_t dtype, const mgemm_cfg *cfg, bool model_may_launch,
                  CallPlan &cp);
// The S partial products of a split plan into W (at least S*m*n elements) and
// their reduction into C, on stream s.
int32_t launch_splitk_into(const KernelEntry *e, const GemmArgs &a, int32_t dtype, bool al,
                           const SplitPlan &sp, uint8_t *W, hipStream_t s);
// C = beta*C for dtype MGEMM_F64 or MGEMM_F32 (beta == 0 writes zeros).
int32_t scale_c(int32_t dtype, int64_t m, int64_t n, double beta, void *C, int64_t ldc,
                hipStream_t s);
int32_t check_args(int64_t m, int64_t n, int64_t k, double alpha, const void *A, int64_t lda,
                   const void *B, int64_t ldb, const void *C, int64_t ldc, int32_t dtype);
int32_t hip_error(hipError_t e, const char *where);
int32_t set_error(int32_t code, const char *fmt, ...);
size_t elem_size(int32_t dtype);
hipStream_t current_stream();

// Writes a cost-model file (format in model.hip); 0 or an error code.
int32_t model_write(const char *path, int I, int H, int O, const int32_t *out_dtype,
                    const mgemm_cfg *out_cfg, const double *mean, const double *stdv,
                    const float *params, int64_t P);
bool cfg_registered(int32_t dtype, const mgemm_cfg &c);

// s_waitcnt immediate for vmcnt(n) (n < 64), no wait on the other counters.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x70 | 0xF00; }

// Number of work-groups a configuration launches for an m x n output.
inline int64_t tiles_of(int64_t m, int64_t n, const mgemm_cfg &c) {
    return ((m + c.bm - 1) / c.bm) * ((n + c.bn - 1) / c.bn);
}

}  // namespace mgemm
