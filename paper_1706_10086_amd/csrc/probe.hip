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

// ---------------------------------------------------------------------------
// Raw-register probe of the low-precision matrix-core steps used by the split
// path.  Lane l passes its operand registers unchanged and gets its accumulator
// registers back, so a test can recover the lane layout of each instruction.
//   kind 0: v_mfma_f32_32x32x16_bf16  a, b: 8 bf16 per lane;  d: 16 float per lane
//   kind 1: v_mfma_i32_32x32x32_i8    a, b: 16 int8 per lane; d: 16 int32 per lane
//   kind 2: v_mfma_f32_16x16x32_bf16  a, b: 8 bf16 per lane;  d: 4 float per lane
//   kind 3: v_mfma_i32_16x16x64_i8    a, b: 16 int8 per lane; d: 4 int32 per lane
//   kind 4: v_mfma_f32_32x32x64_f8f6f4 with both operands FP8 e4m3 (no block
//           scaling)                    a, b: 32 e4m3 per lane; d: 16 float per lane
// ---------------------------------------------------------------------------
namespace mgemm {
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));

__global__ void probe_raw_kernel(int kind, const uint4 *a, const uint4 *b, uint32_t *d) {
    const int l = threadIdx.x;
    if (kind == 4) {
        const v4i a0 = __builtin_bit_cast(v4i, a[2 * l]), a1 = __builtin_bit_cast(v4i, a[2 * l + 1]);
        const v4i b0 = __builtin_bit_cast(v4i, b[2 * l]), b1 = __builtin_bit_cast(v4i, b[2 * l + 1]);
        const v8i va = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        const v8i vb = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
        v16f acc = {};
        // format codes 0, 0: e4m3 operands; scales 0: the unscaled instruction
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(va, vb, acc, 0, 0, 0, 0, 0, 0);
        for (int r = 0; r < 16; ++r) d[l * 16 + r] = __float_as_uint(acc[r]);
        return;
    }
    const uint4 ua = a[l], ub = b[l];
    if (kind == 0) {
        v16f acc = {};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, ua),
                                                      __builtin_bit_cast(v8bf, ub), acc, 0, 0, 0);
        for (int r = 0; r < 16; ++r) d[l * 16 + r] = __float_as_uint(acc[r]);
    } else if (kind == 1) {
        v16i acc = {};
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(v4i, ua),
                                                    __builtin_bit_cast(v4i, ub), acc, 0, 0, 0);
        for (int r = 0; r < 16; ++r) d[l * 16 + r] = (uint32_t)acc[r];
    } else if (kind == 2) {
        v4f acc = {};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, ua),
                                                      __builtin_bit_cast(v8bf, ub), acc, 0, 0, 0);
        for (int r = 0; r < 4; ++r) d[l * 16 + r] = __float_as_uint(acc[r]);
    } else {
        v4i acc = {};
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(v4i, ua),
                                                    __builtin_bit_cast(v4i, ub), acc, 0, 0, 0);
        for (int r = 0; r < 4; ++r) d[l * 16 + r] = (uint32_t)acc[r];
    }
}
}  // namespace mgemm

// a, b: 64 x 16 bytes (one 16-byte operand register group per lane; 64 x 32 for
// kind 4); d: 64 x 16 32-bit words (accumulator element r of lane l at d[16 l + r]).
extern "C" int32_t mgemm_probe_mfma_raw(int32_t kind, const void *a, const void *b, void *d,
                                        void *stream) {
    if (kind < 0 || kind > 4) return mgemm::set_error(-1, "kind must be 0..4");
    if (!a || !b || !d) return mgemm::set_error(-2, "NULL buffer");
    hipLaunchKernelGGL(mgemm::probe_raw_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, kind,
                       (const uint4 *)a, (const uint4 *)b, (uint32_t *)d);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : mgemm::set_error(MGEMM_ERR_HIP, "probe: %s", hipGetErrorString(e));
}
