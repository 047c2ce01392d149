// gemm_ex_noalloc: gemm_ex for FP64 and FP32 without any device allocation, for
// callers that cannot allocate (code under graph capture, tight serving loops).
#include <mutex>

#include "mgemm_internal.h"

namespace mgemm {

// ---------------------------------------------------------------------------
// gemm_ex without allocation: the split-k planes live in `scratch`, a
// file-scope device array (one copy per GPU, held until the process ends).  Its
// device address is looked up once per device (hipGetSymbolAddress with that
// device current, on the entry point's first call there with work to do) and only that address
// is used from the host.  Every split-k plan of a 256-CU GPU fits: the ranges
// times the tiles stay below 8 x 256 tiles of 64 x 64 (two-stage ranges) or at
// most 256 tiles of 128 x 128 (three-stage ranges), i.e. below 2^23 partial
// elements, 64 MiB of FP64; a plan beyond that (a GPU with more compute units)
// is refused.  Every call on a GPU shares its copy: calls that overlap on one
// GPU (on different streams, or from several threads) race on it.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __attribute__((aligned(256))) uint8_t scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mtx;
static uint8_t *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {nullptr};

// The current device's copy of `scratch` (its device address).
static int32_t scratch_on_device(uint8_t **out) {
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return hip_error(he, "scratch: hipGetDevice");
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return set_error(MGEMM_ERR_HIP, "scratch: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (he != hipSuccess || !p) {
            (void)hipGetLastError();
            return hip_error(he != hipSuccess ? he : hipErrorInvalidSymbol,
                             "scratch: hipGetSymbolAddress");
        }
        g_scratch_ptr[dev] = (uint8_t *)p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

static int32_t gemm_noalloc_impl(int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                                 int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                                 int64_t ldc, int32_t dtype, const mgemm_cfg *cfg, void *stream) {
    set_error(0, "%s", "");
    int32_t rc = check_args(m, n, k, alpha, A, lda, B, ldb, C, ldc, dtype);
    if (rc) return rc;
    if (dtype != MGEMM_F64 && dtype != MGEMM_F32)
        return set_error(-12, "gemm_ex_noalloc takes MGEMM_F64 or MGEMM_F32 (the emulated "
                              "dtypes need the library workspace)");
    hipStream_t s = stream ? (hipStream_t)stream : current_stream();
    if (m == 0 || n == 0) return 0;
    if (k == 0 || alpha == 0.0) return scale_c(dtype, m, n, beta, C, ldc, s);
    // the scratch address of this device (looked up on the first call with work)
    uint8_t *W = nullptr;
    rc = scratch_on_device(&W);
    if (rc) return rc;
    GemmArgs a{m, n, k, alpha, beta, A, lda, B, ldb, C, ldc};
    CallPlan cp;
    rc = plan_call(a, dtype, cfg, false, cp);
    if (rc) return rc;
    if (cp.main_rows > 0) {
        // the rows that fill whole rounds run whole, the tail with k cut
        const GemmArgs t = rows_from(a, cp.main_rows, elem_size(dtype));
        const size_t need = (size_t)cp.sp.S * t.m * t.n * elem_size(dtype);
        if (need > SCRATCH_BYTES)
            return set_error(MGEMM_ERR_NOMEM,
                             "gemm_ex_noalloc: split-k needs %zu bytes of scratch, more than its "
                             "%zu-byte maximum", need, SCRATCH_BYTES);
        GemmArgs am = a;
        am.m = cp.main_rows;
        hipError_t he = (cp.al ? cp.e->launch : cp.e->launch_unaligned)(am, s);
        if (he != hipSuccess) return hip_error(he, "gemm launch");
        return launch_splitk_into(cp.e, t, dtype, cp.al, cp.sp, W, s);
    }
    if (cp.sp.S > 1) {
        const size_t need = (size_t)cp.sp.S * a.m * a.n * elem_size(dtype);
        if (need > SCRATCH_BYTES)
            return set_error(MGEMM_ERR_NOMEM,
                             "gemm_ex_noalloc: split-k needs %zu bytes of scratch, more than its "
                             "%zu-byte maximum", need, SCRATCH_BYTES);
        return launch_splitk_into(cp.e, a, dtype, cp.al, cp.sp, W, s);
    }
    hipError_t he = (cp.al ? cp.e->launch : cp.e->launch_unaligned)(a, s);
    if (he != hipSuccess) return hip_error(he, "gemm launch");
    return 0;
}

}  // namespace mgemm

using namespace mgemm;

extern "C" int32_t gemm_ex_noalloc(int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                                   int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                                   int64_t ldc, int32_t dtype, const mgemm_cfg *cfg, void *stream) {
    return gemm_noalloc_impl(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, dtype, cfg, stream);
}
