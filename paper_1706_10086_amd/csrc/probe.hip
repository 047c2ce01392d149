// One matrix-core step on a single wave, for checking the fragment layout that
// the tiled kernels assume: lane l supplies A[l%16][l/16] and B[l/16][l%16] and
// receives column l%16 of D; with q = l/16, accumulator element r holds row
// q + 4r for FP64 and row 4q + r for FP32.
#include "mgemm_internal.h"

namespace mgemm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void probe_f64(const double *A, const double *B, double *D) {
    const int l = threadIdx.x;
    v4d acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(l % 16) * 4 + l / 16], B[(l / 16) * 16 + l % 16],
                                               acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) D[(l / 16 + 4 * r) * 16 + l % 16] = acc[r];
}

__global__ void probe_f32(const float *A, const float *B, float *D) {
    const int l = threadIdx.x;
    v4f acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[(l % 16) * 4 + l / 16], B[(l / 16) * 16 + l % 16],
                                               acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) D[(4 * (l / 16) + r) * 16 + l % 16] = acc[r];
}

int32_t set_error(int32_t code, const char *fmt, ...);

}  // namespace mgemm

using namespace mgemm;

// A is 16x4, B is 4x16, D is 16x16, all row-major device buffers.
extern "C" int32_t mgemm_probe_mfma(int32_t dtype, const void *A, const void *B, void *D,
                                    void *stream) {
    if (!A || !B || !D) return set_error(-2, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == MGEMM_F64)
        hipLaunchKernelGGL(probe_f64, dim3(1), dim3(64), 0, s, (const double *)A,
                           (const double *)B, (double *)D);
    else if (dtype == MGEMM_F32)
        hipLaunchKernelGGL(probe_f32, dim3(1), dim3(64), 0, s, (const float *)A,
                           (const float *)B, (float *)D);
    else
        return set_error(-1, "probe supports F64 and F32");
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : set_error(MGEMM_ERR_HIP, "probe: %s", hipGetErrorString(e));
}
