// The learned tile-configuration cost model: a 3-layer FP32 MLP trained and
// evaluated by the library's own kernels.
//
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3
//   loss = sum M (y - t)^2 / sum M                (masked mean square)
//   Adam update of all parameters (Kingma and Ba, ICLR 2015, Algorithm 1)
//
// Parameters are one flat FP32 vector W1, b1, W2, b2, W3, b3 (row-major).  The
// training set (rows of x, targets t, mask M) lives on the device; one training
// step (forward, loss, backward, Adam) is captured once into a HIP graph and
// replayed per step.  Every reduction runs in a fixed order, so training is
// deterministic.
#include <math.h>

#include <vector>

#include "mgemm_internal.h"

namespace mgemm {

int32_t set_error(int32_t code, const char *fmt, ...);
hipStream_t current_stream();

constexpr int MLP_MAX_DIM = 4096;

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
// Z = X W^T + b (B x O) and A = relu(Z) (or Z); thread per output element, the
// sum over i in increasing order.
__global__ void __launch_bounds__(256)
mlp_fwd_kernel(const float *__restrict__ X, int64_t B, int I, const float *__restrict__ W,
               const float *__restrict__ b, int O, float *__restrict__ Z, float *__restrict__ A,
               int relu) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= B * O) return;
    const int64_t r = idx / O;
    const int o = (int)(idx - r * O);
    const float *x = X + r * I;
    const float *w = W + (int64_t)o * I;
    float z = b[o];
    for (int i = 0; i < I; ++i) z = fmaf(x[i], w[i], z);
    if (Z) Z[idx] = z;
    A[idx] = relu ? fmaxf(z, 0.0f) : z;
}

// Masked mean square loss: dY = 2 M (Y - T) / sum M, loss = sum M (Y - T)^2 / sum M.
// One 256-thread block; also advances the Adam step counter.
__global__ void __launch_bounds__(256)
mlp_loss_kernel(const float *__restrict__ Y, const float *__restrict__ T,
                const float *__restrict__ M, int64_t n, float *__restrict__ dY,
                float *__restrict__ loss, int *step) {
    __shared__ float s_cnt[256], s_sq[256];
    const int tid = threadIdx.x;
    float cnt = 0.0f, sq = 0.0f;
    for (int64_t i = tid; i < n; i += 256) {
        const float d = Y[i] - T[i];
        cnt += M[i];
        sq = fmaf(M[i] * d, d, sq);
    }
    s_cnt[tid] = cnt;
    s_sq[tid] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            s_cnt[tid] += s_cnt[tid + s];
            s_sq[tid] += s_sq[tid + s];
        }
        __syncthreads();
    }
    const float total = s_cnt[0] > 0.0f ? s_cnt[0] : 1.0f;
    const float scale = 2.0f / total;
    for (int64_t i = tid; i < n; i += 256) dY[i] = scale * M[i] * (Y[i] - T[i]);
    if (tid == 0) {
        *loss = s_sq[0] / total;
        if (step) *step += 1;
    }
}

// dZprev = (dZ W) * (Zprev > 0): dZ is B x O, W is O x I, result B x I.
__global__ void __launch_bounds__(256)
mlp_bwd_dx_kernel(const float *__restrict__ dZ, int64_t B, int O, const float *__restrict__ W,
                  int I, const float *__restrict__ Zprev, float *__restrict__ dZprev) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= B * I) return;
    const int64_t r = idx / I;
    const int i = (int)(idx - r * I);
    const float *d = dZ + r * O;
    float s = 0.0f;
    for (int o = 0; o < O; ++o) s = fmaf(d[o], W[(int64_t)o * I + i], s);
    dZprev[idx] = Zprev[idx] > 0.0f ? s : 0.0f;
}

// gW = dZ^T Aprev (O x I) and gb = column sums of dZ; thread per (o, i) and one
// thread per o for the bias, the sum over rows in increasing order.
__global__ void __launch_bounds__(256)
mlp_bwd_dw_kernel(const float *__restrict__ dZ, int64_t B, int O, const float *__restrict__ Aprev,
                  int I, float *__restrict__ gW, float *__restrict__ gb) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nw = (int64_t)O * I;
    if (idx < nw) {
        const int o = (int)(idx / I), i = (int)(idx % I);
        float s = 0.0f;
        for (int64_t r = 0; r < B; ++r) s = fmaf(dZ[r * O + o], Aprev[r * I + i], s);
        gW[idx] = s;
    } else if (idx < nw + O) {
        const int o = (int)(idx - nw);
        float s = 0.0f;
        for (int64_t r = 0; r < B; ++r) s += dZ[r * O + o];
        gb[o] = s;
    }
}

// Adam at the step number held in *step (already advanced for this step).
__global__ void __launch_bounds__(256)
mlp_adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                const int *step) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float t = (float)*step;
    const float bc1 = 1.0f - powf(b1, t);
    const float bc2 = 1.0f - powf(b2, t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Index of the largest Y[r, c] with M[r, c] != 0 (lowest index on ties; -1 if
// no entry is allowed).
__global__ void __launch_bounds__(256)
mlp_argmax_kernel(const float *__restrict__ Y, const float *__restrict__ M, int64_t B, int O,
                  int32_t *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= B) return;
    int best = -1;
    float bv = 0.0f;
    for (int c = 0; c < O; ++c) {
        if (M[r * O + c] == 0.0f) continue;
        const float y = Y[r * O + c];
        if (best < 0 || y > bv) {
            best = c;
            bv = y;
        }
    }
    out[r] = best;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct Mlp {
    int I, H, O;
    int64_t P;
    float *par = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int *step = nullptr;
    float *loss = nullptr;
    // training data and activations (rows B)
    int64_t B = 0;
    float *X = nullptr, *T = nullptr, *M = nullptr;
    float *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *y = nullptr;
    float *dy = nullptr, *dz2 = nullptr, *dz1 = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    float g_lr = 0, g_b1 = 0, g_b2 = 0, g_eps = 0;   // hyper-parameters baked in the graph

    float *W1() { return par; }
    float *b1() { return par + (int64_t)H * I; }
    float *W2() { return b1() + H; }
    float *b2() { return W2() + (int64_t)H * H; }
    float *W3() { return b2() + H; }
    float *b3() { return W3() + (int64_t)O * H; }
    float *gW1() { return grad; }
    float *gb1() { return grad + (int64_t)H * I; }
    float *gW2() { return gb1() + H; }
    float *gb2() { return gW2() + (int64_t)H * H; }
    float *gW3() { return gb2() + H; }
    float *gb3() { return gW3() + (int64_t)O * H; }
};

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

static void free_data(Mlp *p) {
    float **bufs[] = {&p->X, &p->T, &p->M, &p->z1, &p->h1, &p->z2, &p->h2, &p->y, &p->dy, &p->dz2,
                      &p->dz1};
    // teardown: nothing more can be done about a failure here
    for (float **b : bufs) {
        if (*b) (void)hipFree(*b);
        *b = nullptr;
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->B = 0;
}

static void mlp_forward_launch(Mlp *p, int64_t B, const float *X, float *z1, float *h1, float *z2,
                               float *h2, float *y, hipStream_t s) {
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(nblk(B * p->H)), dim3(256), 0, s, X, B, p->I, p->W1(),
                       p->b1(), p->H, z1, h1, 1);
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(nblk(B * p->H)), dim3(256), 0, s, h1, B, p->H, p->W2(),
                       p->b2(), p->H, z2, h2, 1);
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(nblk(B * p->O)), dim3(256), 0, s, h2, B, p->H, p->W3(),
                       p->b3(), p->O, (float *)nullptr, y, 0);
}

// forward + loss + backward on the training set (gradients into p->grad)
static void mlp_grad_launch(Mlp *p, hipStream_t s, bool count_step) {
    const int64_t B = p->B;
    const int I = p->I, H = p->H, O = p->O;
    mlp_forward_launch(p, B, p->X, p->z1, p->h1, p->z2, p->h2, p->y, s);
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, p->y, p->T, p->M, B * O, p->dy,
                       p->loss, count_step ? p->step : (int *)nullptr);
    hipLaunchKernelGGL(mlp_bwd_dw_kernel, dim3(nblk((int64_t)O * H + O)), dim3(256), 0, s, p->dy, B,
                       O, p->h2, H, p->gW3(), p->gb3());
    hipLaunchKernelGGL(mlp_bwd_dx_kernel, dim3(nblk(B * H)), dim3(256), 0, s, p->dy, B, O, p->W3(),
                       H, p->z2, p->dz2);
    hipLaunchKernelGGL(mlp_bwd_dw_kernel, dim3(nblk((int64_t)H * H + H)), dim3(256), 0, s, p->dz2,
                       B, H, p->h1, H, p->gW2(), p->gb2());
    hipLaunchKernelGGL(mlp_bwd_dx_kernel, dim3(nblk(B * H)), dim3(256), 0, s, p->dz2, B, H, p->W2(),
                       H, p->z1, p->dz1);
    hipLaunchKernelGGL(mlp_bwd_dw_kernel, dim3(nblk((int64_t)H * I + H)), dim3(256), 0, s, p->dz1,
                       B, H, p->X, I, p->gW1(), p->gb1());
}

static int32_t hip_err(hipError_t e, const char *w) {
    return set_error(MGEMM_ERR_HIP, "%s: %s", w, hipGetErrorString(e));
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int32_t mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, const float *init_params,
                   void **handle) {
    if (!handle) return set_error(-5, "handle is NULL");
    *handle = nullptr;
    if (in_dim < 1 || in_dim > MLP_MAX_DIM) return set_error(-1, "in_dim out of range");
    if (hidden < 1 || hidden > MLP_MAX_DIM) return set_error(-2, "hidden out of range");
    if (out_dim < 1 || out_dim > MLP_MAX_DIM) return set_error(-3, "out_dim out of range");
    if (!init_params) return set_error(-4, "init_params is NULL");
    Mlp *p = new Mlp();
    p->I = in_dim;
    p->H = hidden;
    p->O = out_dim;
    p->P = (int64_t)hidden * in_dim + hidden + (int64_t)hidden * hidden + hidden +
           (int64_t)out_dim * hidden + out_dim;
    const size_t pb = (size_t)p->P * sizeof(float);
    hipError_t e = hipMalloc((void **)&p->par, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&p->grad, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&p->m, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&p->v, pb);
    if (e == hipSuccess) e = hipMalloc((void **)&p->step, 256);
    if (e == hipSuccess) e = hipMalloc((void **)&p->loss, 256);
    if (e != hipSuccess) {
        mlp_destroy(p);
        return set_error(MGEMM_ERR_NOMEM, "mlp: parameter buffers");
    }
    int32_t rc = mlp_set_params(p, init_params);
    if (rc) {
        mlp_destroy(p);
        return rc;
    }
    *handle = p;
    return 0;
}

int64_t mlp_param_count(void *handle) {
    return handle ? ((Mlp *)handle)->P : -1;
}

int32_t mlp_set_params(void *handle, const float *params) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (!params) return set_error(-2, "params is NULL");
    const size_t pb = (size_t)p->P * sizeof(float);
    hipStream_t s = current_stream();
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(p->par, params, pb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(p->m, 0, pb, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->v, 0, pb, s);
    if (e == hipSuccess) e = hipMemsetAsync(p->step, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? 0 : hip_err(e, "mlp_set_params");
}

int32_t mlp_get_params(void *handle, float *params) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (!params) return set_error(-2, "params is NULL");
    hipError_t e = hipStreamSynchronize(current_stream());
    if (e == hipSuccess) e = hipMemcpy(params, p->par, (size_t)p->P * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? 0 : hip_err(e, "mlp_get_params");
}

int32_t mlp_set_data(void *handle, int64_t rows, const float *X, const float *T, const float *M) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (rows < 1) return set_error(-2, "rows < 1");
    if (!X) return set_error(-3, "X is NULL");
    if (!T) return set_error(-4, "T is NULL");
    if (!M) return set_error(-5, "M is NULL");
    hipError_t se = hipStreamSynchronize(current_stream());
    if (se != hipSuccess) return hip_err(se, "mlp_set_data");
    free_data(p);
    const int64_t B = rows;
    struct { float **dst; int64_t n; } bufs[] = {
        {&p->X, B * p->I}, {&p->T, B * p->O}, {&p->M, B * p->O}, {&p->z1, B * p->H},
        {&p->h1, B * p->H}, {&p->z2, B * p->H}, {&p->h2, B * p->H}, {&p->y, B * p->O},
        {&p->dy, B * p->O}, {&p->dz2, B * p->H}, {&p->dz1, B * p->H}};
    for (auto &b : bufs) {
        if (hipMalloc((void **)b.dst, (size_t)b.n * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            *b.dst = nullptr;
            free_data(p);
            return set_error(MGEMM_ERR_NOMEM, "mlp: training buffers for %lld rows", (long long)rows);
        }
    }
    hipError_t e = hipMemcpy(p->X, X, (size_t)B * p->I * sizeof(float), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->T, T, (size_t)B * p->O * sizeof(float), hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->M, M, (size_t)B * p->O * sizeof(float), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
        free_data(p);
        return hip_err(e, "mlp_set_data");
    }
    p->B = B;
    return 0;
}

int32_t mlp_loss_grad(void *handle, float *loss, float *grad) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (p->B == 0) return set_error(MGEMM_ERR_PLAN, "mlp: no training data");
    hipStream_t s = current_stream();
    mlp_grad_launch(p, s, false);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && loss) e = hipMemcpy(loss, p->loss, sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess && grad)
        e = hipMemcpy(grad, p->grad, (size_t)p->P * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? 0 : hip_err(e, "mlp_loss_grad");
}

int32_t mlp_train(void *handle, int32_t steps, float lr, float beta1, float beta2, float eps,
                  float *last_loss) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (steps < 0) return set_error(-2, "steps < 0");
    if (!(lr > 0.0f)) return set_error(-3, "lr must be positive");
    if (!(beta1 >= 0.0f && beta1 < 1.0f)) return set_error(-4, "beta1 outside [0,1)");
    if (!(beta2 >= 0.0f && beta2 < 1.0f)) return set_error(-5, "beta2 outside [0,1)");
    if (!(eps > 0.0f)) return set_error(-6, "eps must be positive");
    if (p->B == 0) return set_error(MGEMM_ERR_PLAN, "mlp: no training data");
    hipStream_t s = current_stream();
    hipError_t e = hipSuccess;
    // one training step, captured once per hyper-parameter set
    if (!p->exec || p->g_lr != lr || p->g_b1 != beta1 || p->g_b2 != beta2 || p->g_eps != eps) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_err(e, "mlp: capture stream");
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            mlp_grad_launch(p, cs, true);
            hipLaunchKernelGGL(mlp_adam_kernel, dim3(nblk(p->P)), dim3(256), 0, cs, p->par, p->grad,
                               p->m, p->v, p->P, lr, beta1, beta2, eps, (const int *)p->step);
            e = hipStreamEndCapture(cs, &p->graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return hip_err(e, "mlp: training graph");
        p->g_lr = lr;
        p->g_b1 = beta1;
        p->g_b2 = beta2;
        p->g_eps = eps;
    }
    for (int i = 0; i < steps && e == hipSuccess; ++i) e = hipGraphLaunch(p->exec, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && last_loss) e = hipMemcpy(last_loss, p->loss, sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? 0 : hip_err(e, "mlp_train");
}

int32_t mlp_forward(void *handle, int64_t rows, const float *X, float *Y) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (rows < 0) return set_error(-2, "rows < 0");
    if (rows == 0) return 0;
    if (!X) return set_error(-3, "X is NULL");
    if (!Y) return set_error(-4, "Y is NULL");
    float *tmp = nullptr;
    const int64_t B = rows;
    hipError_t e = hipMalloc((void **)&tmp, (size_t)B * p->H * 2 * sizeof(float));
    if (e != hipSuccess) return set_error(MGEMM_ERR_NOMEM, "mlp_forward: scratch");
    hipStream_t s = current_stream();
    mlp_forward_launch(p, B, X, (float *)nullptr, tmp, (float *)nullptr, tmp + B * p->H, Y, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e == hipSuccess ? 0 : hip_err(e, "mlp_forward");
}

int32_t mlp_predict(void *handle, int64_t rows, const float *X, const float *M, int32_t *idx) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (rows < 0) return set_error(-2, "rows < 0");
    if (rows == 0) return 0;
    if (!X) return set_error(-3, "X is NULL");
    if (!M) return set_error(-4, "M is NULL");
    if (!idx) return set_error(-5, "idx is NULL");
    float *y = nullptr;
    hipError_t e = hipMalloc((void **)&y, (size_t)rows * p->O * sizeof(float));
    if (e != hipSuccess) return set_error(MGEMM_ERR_NOMEM, "mlp_predict: scratch");
    int32_t rc = mlp_forward(p, rows, X, y);
    if (rc == 0) {
        hipStream_t s = current_stream();
        hipLaunchKernelGGL(mlp_argmax_kernel, dim3(nblk(rows)), dim3(256), 0, s, y, M, rows, p->O,
                           idx);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_err(e, "mlp_predict");
    }
    (void)hipFree(y);
    return rc;
}

int32_t mlp_save(void *handle, const char *path, const int32_t *out_dtype,
                 const mgemm_cfg *out_cfg, const double *feat_mean, const double *feat_std) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (!path) return set_error(-2, "path is NULL");
    if (!out_dtype) return set_error(-3, "out_dtype is NULL");
    if (!out_cfg) return set_error(-4, "out_cfg is NULL");
    if (!feat_mean) return set_error(-5, "feat_mean is NULL");
    if (!feat_std) return set_error(-6, "feat_std is NULL");
    if (p->I != 6)
        return set_error(MGEMM_ERR_MODEL, "model files hold networks of 6 inputs, not %d", p->I);
    for (int o = 0; o < p->O; ++o)
        if (!cfg_registered(out_dtype[o], out_cfg[o]))
            return set_error(MGEMM_ERR_MODEL, "output %d names a configuration not registered", o);
    std::vector<float> par((size_t)p->P);
    const int32_t rc = mlp_get_params(p, par.data());
    if (rc) return rc;
    return model_write(path, p->I, p->H, p->O, out_dtype, out_cfg, feat_mean, feat_std, par.data(),
                       p->P);
}

int32_t mlp_destroy(void *handle) {
    Mlp *p = (Mlp *)handle;
    if (!p) return 0;
    const hipError_t e = hipStreamSynchronize(current_stream());   // work that uses p
    free_data(p);
    float **bufs[] = {&p->par, &p->grad, &p->m, &p->v, &p->loss};
    for (float **b : bufs)
        if (*b) (void)hipFree(*b);
    if (p->step) (void)hipFree(p->step);
    delete p;
    return e == hipSuccess ? 0 : hip_err(e, "mlp_destroy: stream synchronize");
}

}  // extern "C"
