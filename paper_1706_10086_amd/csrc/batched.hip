// Batched GEMM: many independent problems C_i = alpha_i A_i B_i + beta_i C_i.
//
//  * gemm_batched            one gemm_ex launch per problem (the per-problem
//                            baseline).
//  * gemm_batched_plan_*     problems are grouped by tile configuration (chosen
//                            per problem, or given by the caller) and by row
//                            alignment into buckets; each bucket's problems are
//                            ordered by decreasing work and numbered tile by tile
//                            into one work list, copied to the device once; one
//                            persistent kernel per bucket (grid = resident
//                            work-groups of the whole GPU) pulls tiles from an
//                            atomic counter.  A counter-reset kernel and the
//                            bucket kernels (as parallel branches) are captured
//                            once into a HIP graph; executing the plan is one
//                            hipGraphLaunch.  Each tile runs the same code as
//                            gemm_ex with the same configuration, so results are
//                            bitwise identical to per-problem gemm_ex calls.
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
    int align;                        // 0: aligned rows, 1: any rows
    std::vector<BatchProblem> probs;
    int64_t total_tiles = 0;
    int grid = 0;
    size_t offset = 0;                // byte offset of the descriptors in dev
};

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
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->dev) hipFree(p->dev);
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
    hipGetDevice(&p->device);

    // bucket by (configuration, alignment)
    std::map<std::pair<const KernelEntry *, int>, size_t> index;
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
        if (!e) {
            plan_free(p);
            return err ? err : set_error(MGEMM_ERR_NOCONFIG, "problem %lld: no configuration",
                                         (long long)i);
        }
        const int al = rows_aligned(A[i], lda[i], B[i], ldb[i], dtype) ? 0 : 1;
        auto key = std::make_pair(e, al);
        auto it = index.find(key);
        if (it == index.end()) {
            index[key] = p->buckets.size();
            Bucket b;
            b.entry = e;
            b.align = al;
            p->buckets.push_back(b);
            it = index.find(key);
        }
        BatchProblem bp;
        bp.g = GemmArgs{m[i], n[i], k[i], alpha[i], beta[i], A[i], lda[i], B[i], ldb[i], C[i], ldc[i]};
        bp.tile0 = 0;
        bp.tiles_n = (n[i] + e->cfg.bn - 1) / e->cfg.bn;
        p->buckets[it->second].probs.push_back(bp);
        p->flops += 2.0 * (double)m[i] * (double)n[i] * (double)k[i];
    }

    int cus = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (cus <= 0) cus = 1;
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
        const int64_t resident = (int64_t)cus * b.entry->batched_occupancy[b.align]();
        b.grid = (int)std::min<int64_t>(resident, t);
        b.offset = bytes;
        bytes += (b.probs.size() * sizeof(BatchProblem) + 255) / 256 * 256;
    }
    const size_t counters_off = bytes;
    const int nb = (int)p->buckets.size();
    bytes += (size_t)std::max(nb, 1) * sizeof(unsigned long long);

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
        hipLaunchKernelGGL(reset_counters_kernel, dim3((unsigned)((std::max(nb, 1) + 63) / 64)),
                           dim3(64), 0, cs, counters, std::max(nb, 1));
        hipEventRecord(start, cs);
        for (int b = 0; b < nb; ++b) {
            Bucket &bk = p->buckets[b];
            hipStreamWaitEvent(branch[b], start, 0);
            hipError_t le = bk.entry->batched[bk.align](
                (const BatchProblem *)(p->dev + bk.offset), (int)bk.probs.size(), bk.total_tiles,
                counters + b, bk.grid, branch[b]);
            if (le != hipSuccess && rc == 0) rc = hip_fail(le, "plan: bucket launch");
            hipEventRecord(done[b], branch[b]);
            hipStreamWaitEvent(cs, done[b], 0);
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
        if (done[b]) hipEventDestroy(done[b]);
        if (branch[b]) hipStreamDestroy(branch[b]);
    }
    if (start) hipEventDestroy(start);
    if (cs) hipStreamDestroy(cs);
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
    hipStreamSynchronize(p->stream);
    plan_free(p);
    return 0;
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
