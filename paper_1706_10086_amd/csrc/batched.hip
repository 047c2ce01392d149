// Batched GEMM: many independent problems C_i = alpha_i A_i B_i + beta_i C_i.
//
//  * gemm_batched            one gemm_ex launch per problem (the per-problem
//                            baseline).
//  * gemm_batched_plan_*     problems are grouped by tile configuration (chosen
//                            per problem, or given by the caller) into buckets;
//                            each bucket's problems are ordered by decreasing
//                            work and dealt into work lists (one per XCD; a map
//                            entry names a problem, tile row and tile column),
//                            copied to the device once; one persistent kernel
//                            per bucket (grid = resident work-groups of the whole
//                            GPU) pulls tiles from atomic counters.  A
//                            counter-reset kernel and the bucket kernels (as
//                            parallel branches) are captured once into a HIP
//                            graph; executing the plan is one hipGraphLaunch.
//                            Each tile runs the same code as gemm_ex with the
//                            same configuration and row alignment, so results
//                            are bitwise identical to per-problem gemm_ex calls.
#include <algorithm>
#include <map>
#include <vector>

#include "mgemm_internal.h"

namespace mgemm {

int32_t set_error(int32_t code, const char *fmt, ...);
int32_t check_args(int64_t m, int64_t n, int64_t k, double alpha, const void *A, int64_t lda,
                   const void *B, int64_t ldb, const void *C, int64_t ldc, int32_t dtype);
const KernelEntry *choose_entry(int32_t dtype, int64_t m, int64_t n, const mgemm_cfg *cfg,
                                int32_t *err);
bool rows_aligned(const void *A, int64_t lda, const void *B, int64_t ldb, int32_t dtype);

static const mgemm_cfg kBatchedDefault = {64, 64, 16, 4, 2, 1, 0};

__global__ void reset_counters_kernel(unsigned long long *c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0ull;
}

struct Bucket {
    const KernelEntry *entry;
    std::vector<BatchProblem> probs;
    int64_t total_tiles = 0;
    int grid = 0;
    size_t offset = 0;                // byte offset of the descriptors in dev
    size_t map_offset = 0;            // byte offset of the tile map in dev (if use_map)
    size_t list_offset = 0;           // byte offset of the list bounds in dev
    bool use_map = false;
    std::vector<uint64_t> map;        // the lists' entries, list after list (host copy)
    std::vector<int64_t> list_off;    // list l holds [list_off[l], list_off[l+1])
};

// Tile maps are built while every bucket's map fits this many bytes in total and
// each entry's fields fit their bit widths; otherwise the kernels search.
constexpr size_t TILE_MAP_MAX_BYTES = (size_t)256 << 20;

// One list per XCD: problems, in decreasing work, are cut into runs of whole
// tile rows of about 1/16 of a list's share of the work, and each run goes to the
// list with the least work so far; a run's tiles share their rows of A (and read
// the same B) in the L2 of the XCD that serves the list.
static void build_lists(Bucket &b) {
    const mgemm_cfg &c = b.entry->cfg;
    double total = 0.0;
    for (const BatchProblem &bp : b.probs)
        total += (double)((bp.g.m + c.bm - 1) / c.bm) * (double)bp.tiles_n * (double)bp.g.k;
    const double piece = std::max(total / (BATCH_LISTS * 16.0), 1.0);
    std::vector<std::vector<uint64_t>> lists(BATCH_LISTS);
    std::vector<double> load(BATCH_LISTS, 0.0);
    for (size_t j = 0; j < b.probs.size(); ++j) {
        const BatchProblem &bp = b.probs[j];
        const int64_t tiles_m = (bp.g.m + c.bm - 1) / c.bm;
        const double row_work = (double)bp.tiles_n * (double)bp.g.k;
        const int64_t rows = std::max<int64_t>(1, (int64_t)(piece / row_work));
        for (int64_t tm0 = 0; tm0 < tiles_m; tm0 += rows) {
            const int64_t tm1 = std::min(tiles_m, tm0 + rows);
            const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int64_t tm = tm0; tm < tm1; ++tm)
                for (int64_t tn = 0; tn < bp.tiles_n; ++tn)
                    lists[l].push_back(tile_map_entry(j, (uint64_t)tm, (uint64_t)tn));
            load[l] += (double)(tm1 - tm0) * row_work;
        }
    }
    b.map.clear();
    b.list_off.assign(1, 0);
    for (const auto &li : lists) {
        b.map.insert(b.map.end(), li.begin(), li.end());
        b.list_off.push_back((int64_t)b.map.size());
    }
}

struct Plan {
    int device = 0;
    int32_t dtype = 0;
    hipStream_t stream = nullptr;     // execution stream
    std::vector<Bucket> buckets;
    uint8_t *dev = nullptr;           // descriptors + counters
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t count = 0;
    double flops = 0.0;
};

static void plan_free(Plan *p) {
    if (!p) return;
    // teardown: nothing more can be done about a failure here
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

static int32_t hip_fail(hipError_t e, const char *what) {
    return set_error(MGEMM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int32_t gemm_batched(int64_t count, const int64_t *m, const int64_t *n, const int64_t *k,
                     const double *alpha, const void *const *A, const int64_t *lda,
                     const void *const *B, const int64_t *ldb, const double *beta,
                     void *const *C, const int64_t *ldc, int32_t dtype) {
    if (count < 0) return set_error(-1, "count < 0");
    if (count == 0) return 0;
    if (!m) return set_error(-2, "m is NULL");
    if (!n) return set_error(-3, "n is NULL");
    if (!k) return set_error(-4, "k is NULL");
    if (!alpha) return set_error(-5, "alpha is NULL");
    if (!A) return set_error(-6, "A is NULL");
    if (!lda) return set_error(-7, "lda is NULL");
    if (!B) return set_error(-8, "B is NULL");
    if (!ldb) return set_error(-9, "ldb is NULL");
    if (!beta) return set_error(-10, "beta is NULL");
    if (!C) return set_error(-11, "C is NULL");
    if (!ldc) return set_error(-12, "ldc is NULL");
    for (int64_t i = 0; i < count; ++i) {
        int32_t rc = check_args(m[i], n[i], k[i], alpha[i], A[i], lda[i], B[i], ldb[i], C[i],
                                ldc[i], dtype);
        if (rc) return set_error(rc, "problem %lld: argument %d invalid", (long long)i, -rc);
    }
    for (int64_t i = 0; i < count; ++i) {
        int32_t rc = gemm_ex(m[i], n[i], k[i], alpha[i], A[i], lda[i], B[i], ldb[i], beta[i], C[i],
                             ldc[i], dtype, nullptr, nullptr);
        if (rc) return rc;
    }
    return 0;
}

int32_t gemm_batched_plan_create(int64_t count, const int64_t *m, const int64_t *n,
                                 const int64_t *k, const double *alpha, const void *const *A,
                                 const int64_t *lda, const void *const *B, const int64_t *ldb,
                                 const double *beta, void *const *C, const int64_t *ldc,
                                 int32_t dtype, const mgemm_cfg *cfgs, void *stream,
                                 void **plan_out) {
    if (!plan_out) return set_error(-16, "plan is NULL");
    *plan_out = nullptr;
    if (count < 0) return set_error(-1, "count < 0");
    if (count > 0 && (!m || !n || !k || !alpha || !A || !lda || !B || !ldb || !beta || !C || !ldc))
        return set_error(-2, "a problem array is NULL");
    if (dtype != MGEMM_F64 && dtype != MGEMM_F32)
        return set_error(-13, "batched plans take MGEMM_F64 or MGEMM_F32");
    for (int64_t i = 0; i < count; ++i) {
        int32_t rc = check_args(m[i], n[i], k[i], alpha[i], A[i], lda[i], B[i], ldb[i], C[i],
                                ldc[i], dtype);
        if (rc) return set_error(rc, "problem %lld: argument %d invalid", (long long)i, -rc);
    }

    Plan *p = new Plan();
    p->dtype = dtype;
    p->stream = (hipStream_t)stream;
    p->count = count;
    {
        hipError_t de = hipGetDevice(&p->device);
        if (de != hipSuccess) {
            plan_free(p);
            return hip_fail(de, "plan: no current device");
        }
    }

    // bucket by configuration
    std::map<const KernelEntry *, size_t> index;
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] == 0 || n[i] == 0) continue;
        if (k[i] == 0 || alpha[i] == 0.0) {
            plan_free(p);
            return set_error(MGEMM_ERR_PLAN,
                             "problem %lld: k == 0 or alpha == 0 is not supported in a plan",
                             (long long)i);
        }
        int32_t err = 0;
        // without caller configurations every problem of a plan uses the 64 x 64 x 16
        // four-wave tile: in a batch the other problems supply the parallelism, and
        // one bucket beat mixtures of tile sizes on the uneven batched workload
        // (28.2 vs 18.8 TFLOP/s with the single-GEMM choice, MI355X)
        const KernelEntry *e =
            choose_entry(dtype, m[i], n[i], cfgs ? &cfgs[i] : &kBatchedDefault, &err);
        if (!e || !e->batched) {
            plan_free(p);
            if (cfgs)
                return set_error(-14, "problem %lld: configuration %dx%dx%d w%d e%d d%d o%d is %s",
                                 (long long)i, cfgs[i].bm, cfgs[i].bn, cfgs[i].bk, cfgs[i].waves,
                                 cfgs[i].elems_per_thread, cfgs[i].double_buffer,
                                 cfgs[i].occupancy,
                                 e ? "not available in batched plans" : "not registered");
            return err ? err : set_error(MGEMM_ERR_NOCONFIG, "problem %lld: no configuration",
                                         (long long)i);
        }
        auto it = index.find(e);
        if (it == index.end()) {
            index[e] = p->buckets.size();
            Bucket b;
            b.entry = e;
            p->buckets.push_back(b);
            it = index.find(e);
        }
        BatchProblem bp;
        bp.g = GemmArgs{m[i], n[i], k[i], alpha[i], beta[i], A[i], lda[i], B[i], ldb[i], C[i], ldc[i]};
        bp.tile0 = 0;
        bp.tiles_n = (n[i] + e->cfg.bn - 1) / e->cfg.bn;
        bp.aligned = rows_aligned(A[i], lda[i], B[i], ldb[i], dtype) ? 1 : 0;
        p->buckets[it->second].probs.push_back(bp);
        p->flops += 2.0 * (double)m[i] * (double)n[i] * (double)k[i];
    }

    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
        cus <= 0)
        cus = 1;   // a smaller persistent grid is still correct
    size_t bytes = 0;
    for (Bucket &b : p->buckets) {
        const mgemm_cfg &c = b.entry->cfg;
        std::stable_sort(b.probs.begin(), b.probs.end(), [&](const BatchProblem &x,
                                                             const BatchProblem &y) {
            const double wx = (double)((x.g.m + c.bm - 1) / c.bm) * x.tiles_n * (double)x.g.k;
            const double wy = (double)((y.g.m + c.bm - 1) / c.bm) * y.tiles_n * (double)y.g.k;
            return wx > wy;
        });
        int64_t t = 0;
        for (BatchProblem &bp : b.probs) {
            bp.tile0 = t;
            t += ((bp.g.m + c.bm - 1) / c.bm) * bp.tiles_n;
        }
        b.total_tiles = t;
        const int64_t resident = (int64_t)cus * b.entry->batched_occupancy();
        b.grid = (int)std::min<int64_t>(resident, t);
        b.offset = bytes;
        bytes += (b.probs.size() * sizeof(BatchProblem) + 255) / 256 * 256;
    }
    // tile maps (one 8-byte entry per tile, in per-XCD lists) if the fields fit
    // and the total is modest; otherwise one list of tile numbers
    {
        bool fits = true;
        size_t map_bytes = 0;
        for (const Bucket &b : p->buckets) {
            if (b.probs.size() >= ((size_t)1 << TILE_MAP_PROB_BITS)) fits = false;
            for (const BatchProblem &bp : b.probs) {
                const int64_t tiles_m = (bp.g.m + b.entry->cfg.bm - 1) / b.entry->cfg.bm;
                if (tiles_m >= ((int64_t)1 << TILE_MAP_RC_BITS) ||
                    bp.tiles_n >= ((int64_t)1 << TILE_MAP_RC_BITS))
                    fits = false;
            }
            map_bytes += ((size_t)b.total_tiles * sizeof(uint64_t) + 255) / 256 * 256;
        }
        for (Bucket &b : p->buckets) {
            if (fits && map_bytes <= TILE_MAP_MAX_BYTES) {
                b.use_map = true;
                build_lists(b);
                b.map_offset = bytes;
                bytes += (b.map.size() * sizeof(uint64_t) + 255) / 256 * 256;
            } else {
                b.list_off = {0, b.total_tiles};
            }
            b.list_offset = bytes;
            bytes += (b.list_off.size() * sizeof(int64_t) + 255) / 256 * 256;
        }
    }
    const size_t counters_off = bytes;
    const int nb = (int)p->buckets.size();
    const int ncounters = std::max(nb, 1) * BATCH_LISTS;
    bytes += (size_t)ncounters * sizeof(unsigned long long);

    hipError_t he = hipMalloc((void **)&p->dev, bytes);
    if (he != hipSuccess) {
        (void)hipGetLastError();
        p->dev = nullptr;
        plan_free(p);
        return set_error(MGEMM_ERR_NOMEM, "plan: %zu bytes of descriptors not available", bytes);
    }
    for (Bucket &b : p->buckets) {
        he = hipMemcpy(p->dev + b.offset, b.probs.data(), b.probs.size() * sizeof(BatchProblem),
                       hipMemcpyHostToDevice);
        if (he == hipSuccess && b.use_map)
            he = hipMemcpy(p->dev + b.map_offset, b.map.data(), b.map.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice);
        if (he == hipSuccess)
            he = hipMemcpy(p->dev + b.list_offset, b.list_off.data(),
                           b.list_off.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        std::vector<uint64_t>().swap(b.map);
        if (he != hipSuccess) {
            plan_free(p);
            return hip_fail(he, "plan: descriptor copy");
        }
    }
    unsigned long long *counters = (unsigned long long *)(p->dev + counters_off);

    // capture: reset counters, then every bucket kernel on its own branch
    hipStream_t cs = nullptr;
    std::vector<hipStream_t> branch(nb, nullptr);
    std::vector<hipEvent_t> done(nb, nullptr);
    hipEvent_t start = nullptr;
    int32_t rc = 0;
    he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    for (int b = 0; b < nb && he == hipSuccess; ++b) {
        he = hipStreamCreateWithFlags(&branch[b], hipStreamNonBlocking);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&done[b], hipEventDisableTiming);
    }
    if (he == hipSuccess) he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
        hipLaunchKernelGGL(reset_counters_kernel, dim3((unsigned)((ncounters + 63) / 64)),
                           dim3(64), 0, cs, counters, ncounters);
        hipError_t ge = hipEventRecord(start, cs);
        if (ge != hipSuccess && rc == 0) rc = hip_fail(ge, "plan: capture record");
        for (int b = 0; b < nb; ++b) {
            Bucket &bk = p->buckets[b];
            ge = hipStreamWaitEvent(branch[b], start, 0);
            if (ge != hipSuccess && rc == 0) rc = hip_fail(ge, "plan: capture fork");
            hipError_t le = bk.entry->batched(
                (const BatchProblem *)(p->dev + bk.offset),
                bk.use_map ? (const uint64_t *)(p->dev + bk.map_offset) : nullptr,
                (const int64_t *)(p->dev + bk.list_offset), (int)bk.list_off.size() - 1,
                (int)bk.probs.size(), counters + (size_t)b * BATCH_LISTS, bk.grid, branch[b]);
            if (le != hipSuccess && rc == 0) rc = hip_fail(le, "plan: bucket launch");
            ge = hipEventRecord(done[b], branch[b]);
            if (ge == hipSuccess) ge = hipStreamWaitEvent(cs, done[b], 0);
            if (ge != hipSuccess && rc == 0) rc = hip_fail(ge, "plan: capture join");
        }
        hipError_t ce = hipStreamEndCapture(cs, &p->graph);
        if (ce != hipSuccess && rc == 0) rc = hip_fail(ce, "plan: capture");
        if (rc == 0) {
            ce = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            if (ce != hipSuccess) rc = hip_fail(ce, "plan: instantiate");
        }
    } else {
        rc = hip_fail(he, "plan: stream setup");
    }
    for (int b = 0; b < nb; ++b) {
        if (done[b]) (void)hipEventDestroy(done[b]);
        if (branch[b]) (void)hipStreamDestroy(branch[b]);
    }
    if (start) (void)hipEventDestroy(start);
    if (cs) (void)hipStreamDestroy(cs);
    if (rc) {
        plan_free(p);
        return rc;
    }
    *plan_out = p;
    return 0;
}

int32_t gemm_batched_plan_execute(void *plan) {
    Plan *p = (Plan *)plan;
    if (!p || !p->exec) return set_error(MGEMM_ERR_PLAN, "not a plan");
    hipError_t he = hipGraphLaunch(p->exec, p->stream);
    return he == hipSuccess ? 0 : hip_fail(he, "plan execute");
}

int32_t gemm_batched_plan_destroy(void *plan) {
    Plan *p = (Plan *)plan;
    if (!p) return 0;
    const hipError_t he = hipStreamSynchronize(p->stream);   // the plan's last launch
    plan_free(p);
    return he == hipSuccess ? 0 : hip_fail(he, "plan destroy: stream synchronize");
}

int32_t gemm_batched_plan_info(void *plan, int32_t *buckets, int64_t *total_tiles, double *flops) {
    Plan *p = (Plan *)plan;
    if (!p) return set_error(MGEMM_ERR_PLAN, "not a plan");
    int64_t t = 0;
    for (const Bucket &b : p->buckets) t += b.total_tiles;
    if (buckets) *buckets = (int32_t)p->buckets.size();
    if (total_tiles) *total_tiles = t;
    if (flops) *flops = p->flops;
    return 0;
}

}  // extern "C"
