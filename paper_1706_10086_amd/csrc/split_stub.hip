// Placeholder for the split-precision path until its kernels land.
#include "mgemm_internal.h"

namespace mgemm {
int32_t set_error(int32_t code, const char *fmt, ...);

int32_t split_gemm(const GemmArgs &, int32_t, hipStream_t) {
    return set_error(MGEMM_ERR_NOCONFIG, "split-precision path not built");
}
}  // namespace mgemm

extern "C" int32_t mgemm_release_workspace(void) { return 0; }
