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
// replayed per step.  The linear layers' products (forward, the backward
// products and the weight gradients) run on the matrix cores in FP32; every
// reduction runs in a fixed order, so training is deterministic.
#include <math.h>

#include <algorithm>
#include <vector>

#include "tile_gemm.h"

namespace mgemm {

int32_t set_error(int32_t code, const char *fmt, ...);
hipStream_t current_stream();

constexpr int MLP_MAX_DIM = 4096;
constexpr int64_t MLP_MAX_ROWS = (int64_t)1 << 30;

// ---------------------------------------------------------------------------
// The products of the network on the matrix cores.
// ---------------------------------------------------------------------------
// Every linear step -- forward Z = A W^T, backward dA = dZ W and the gradient
// dW = dZ^T A -- is one small product op(P) op(Q) of FP32 matrices, computed by
// mm_kernel with FP32 MFMA (v_mfma_f32_16x16x4_f32, FP32 products and sums) in
// 64 x 64 tiles of the result: four waves of 32 x 32, k in steps of 16 staged in
// LDS, the next step's operands loaded into registers during the current one.
// op(P) is P (row-major, P[m*ldp + k]) or its transpose (P[k*ldp + m]), likewise
// op(Q).  The gradient products reduce over the training rows: their k range is
// cut into blockIdx.z ranges whose partial tiles go to separate planes, added in
// plane order by mm_reduce_kernel, so every sum has a fixed order (training is
// deterministic).  A bias is the weight of a constant input: its gradient is the
// last column of dZ^T [A | 1], the ones column read by the product itself.
constexpr int MM_T = 64;        // result tile (rows and columns)
constexpr int MM_K = 16;        // k per staged step
constexpr int MM_SA = MM_T + 4; // LDS row stride (k-major tiles)

enum MmEpi {
    MM_STORE = 0,       // C = s * acc
    MM_BIAS_RELU = 1,   // Z = acc + bias[n] (stored when Z2 != NULL), C = relu(Z)
    MM_BIAS_LOSS = 2,   // C = Y = acc + bias[n]; D = M (Y - T); per-tile sums of M and M (Y - T)^2
    MM_MASK = 3,        // C = Zp > 0 ? s * acc : 0 (relu derivative of the layer below)
    MM_PARTIAL = 4,     // plane z of C: s * acc over this block's k range
    MM_BIAS = 5,        // C = acc + bias[n]
};

struct MmArgs {
    const float *P;
    int64_t ldp;
    const float *Q;
    int64_t ldq;
    int M, N;
    int64_t K, kchunk;        // k in [z*kchunk, min(K, (z+1)*kchunk)) for blockIdx.z = z
    int ones_col;             // >= 0: column ones_col of op(Q) reads 1 (bias gradient)
    const float *scale;       // non-NULL: s = *scale, else 1
    const float *bias;        // MM_BIAS_*: per column
    const float *Zp;          // MM_MASK: pre-activation with the result's layout
    const float *T, *Mk;      // MM_BIAS_LOSS: targets and mask (result's layout)
    float *C;
    int64_t ldc;
    float *Z2;                // MM_BIAS_RELU: pre-activation out; MM_BIAS_LOSS: D out
    float *part;              // MM_BIAS_LOSS: 2 floats per block (mask sum, square sum)
    int64_t plane;            // MM_PARTIAL: elements per plane
};

template <bool TP, bool TQ, int EPI>
__global__ void __launch_bounds__(256) mm_kernel(MmArgs a) {
    typedef Elem<float> E;
    __shared__ float sP[MM_K * MM_SA];
    __shared__ float sQ[MM_K * MM_SA];
    __shared__ float sRed[2][256];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.x * MM_T, n0 = blockIdx.y * MM_T;
    const int64_t kb = (int64_t)blockIdx.z * a.kchunk;
    const int64_t ke = kb + a.kchunk < a.K ? kb + a.kchunk : a.K;

    // element e = tid + 256 j of a 64 x 16 operand tile: (row r, k c) with the
    // contiguous global index running fastest across threads
    float rp[4], rq[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j;
            int r, c;
            if (TP) { r = e & 63; c = e >> 6; } else { r = e >> 4; c = e & 15; }
            const int64_t gm = m0 + r, gk = k0 + c;
            float v = 0.0f;
            if (gm < a.M && gk < ke) v = TP ? a.P[gk * a.ldp + gm] : a.P[gm * a.ldp + gk];
            rp[j] = v;
            if (TQ) { r = e >> 4; c = e & 15; } else { r = e & 63; c = e >> 6; }
            const int64_t gn = n0 + r, gq = k0 + c;
            float w = 0.0f;
            if (gn < a.N && gq < ke)
                w = gn == a.ones_col ? 1.0f : (TQ ? a.Q[gn * a.ldq + gq] : a.Q[gq * a.ldq + gn]);
            rq[j] = w;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j;
            int r, c;
            if (TP) { r = e & 63; c = e >> 6; } else { r = e >> 4; c = e & 15; }
            sP[c * MM_SA + r] = rp[j];
            if (TQ) { r = e >> 4; c = e & 15; } else { r = e & 63; c = e >> 6; }
            sQ[c * MM_SA + r] = rq[j];
        }
    };

    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0, 0, 0, 0};
    const int l16 = lane & 15, kq = lane >> 4;
    if (kb < ke) load(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += MM_K) {
        __syncthreads();          // the previous step's reads of the tiles are done
        store();
        __syncthreads();
        if (k0 + MM_K < ke) load(k0 + MM_K);
#pragma unroll
        for (int g = 0; g < MM_K / 4; ++g) {
            const int kk = 4 * g + kq;
            float pf[2], qf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) pf[i] = sP[kk * MM_SA + wm * 32 + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < 2; ++j) qf[j] = sQ[kk * MM_SA + wn * 32 + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = E::mma(pf[i], qf[j], acc[i][j]);
        }
    }

    const float s = a.scale ? *a.scale : 1.0f;
    float cnt = 0.0f, sq = 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 32 + j * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + i * 16 + E::out_row(kq, r);
                if (m >= a.M || n >= a.N) continue;
                const float v = acc[i][j][r];
                const int64_t o = (int64_t)m * a.ldc + n;
                if (EPI == MM_STORE) {
                    a.C[o] = s * v;
                } else if (EPI == MM_BIAS_RELU) {
                    const float z = v + a.bias[n];
                    if (a.Z2) a.Z2[o] = z;
                    a.C[o] = fmaxf(z, 0.0f);
                } else if (EPI == MM_BIAS_LOSS) {
                    const float y = v + a.bias[n];
                    const float mk = a.Mk[o];
                    const float d = y - a.T[o];
                    a.C[o] = y;
                    a.Z2[o] = mk * d;
                    cnt += mk;
                    sq = fmaf(mk * d, d, sq);
                } else if (EPI == MM_BIAS) {
                    a.C[o] = v + a.bias[n];
                } else if (EPI == MM_MASK) {
                    a.C[o] = a.Zp[o] > 0.0f ? s * v : 0.0f;
                } else {
                    a.C[(int64_t)blockIdx.z * a.plane + o] = s * v;
                }
            }
        }
    if (EPI == MM_BIAS_LOSS) {
        // this tile's sums, added in a fixed order
        sRed[0][tid] = cnt;
        sRed[1][tid] = sq;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) {
                sRed[0][tid] += sRed[0][tid + h];
                sRed[1][tid] += sRed[1][tid + h];
            }
            __syncthreads();
        }
        if (tid == 0) {
            const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
            a.part[2 * blk] = sRed[0][0];
            a.part[2 * blk + 1] = sRed[1][0];
        }
    }
}

// Sum of the S planes (M x (N + 1) elements each, in plane order) of a gradient
// product dZ^T [A | 1]: columns 0..N-1 to gW (M x N), column N to gb.
__global__ void __launch_bounds__(256)
mm_reduce_kernel(const float *__restrict__ planes, int S, int M, int N, float *__restrict__ gW,
                 float *__restrict__ gb) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t plane = (int64_t)M * (N + 1);
    if (idx >= plane) return;
    float v = planes[idx];
    for (int z = 1; z < S; ++z) v += planes[z * plane + idx];
    const int m = (int)(idx / (N + 1)), n = (int)(idx % (N + 1));
    if (n < N) gW[(int64_t)m * N + n] = v;
    else gb[m] = v;
}

// The loss from the per-tile sums (in tile order): loss = sum M (Y-T)^2 / sum M,
// and the factor 2 / sum M that turns D = M (Y - T) into dL/dY; also advances the
// Adam step counter.
__global__ void __launch_bounds__(256)
mlp_loss_final_kernel(const float *__restrict__ part, int tiles, float *__restrict__ loss,
                      float *__restrict__ scale, int *step) {
    __shared__ float s_cnt[256], s_sq[256];
    const int tid = threadIdx.x;
    float cnt = 0.0f, sq = 0.0f;
    for (int i = tid; i < tiles; i += 256) {
        cnt += part[2 * i];
        sq += part[2 * i + 1];
    }
    s_cnt[tid] = cnt;
    s_sq[tid] = sq;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            s_cnt[tid] += s_cnt[tid + h];
            s_sq[tid] += s_sq[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const float total = s_cnt[0] > 0.0f ? s_cnt[0] : 1.0f;
        *loss = s_sq[0] / total;
        *scale = 2.0f / total;
        if (step) *step += 1;
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
    float *loss = nullptr;    // [0] loss, [1] 2 / sum of the mask
    // training data and activations (rows B)
    int64_t B = 0;
    float *X = nullptr, *T = nullptr, *M = nullptr;
    float *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *y = nullptr;
    float *d = nullptr, *dz2 = nullptr, *dz1 = nullptr;   // d = M (y - t)
    float *planes = nullptr;  // partial gradient planes
    float *part = nullptr;    // per-tile loss sums of the output layer
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
    float **bufs[] = {&p->X, &p->T, &p->M, &p->z1, &p->h1, &p->z2, &p->h2, &p->y, &p->d, &p->dz2,
                      &p->dz1, &p->planes, &p->part};
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

static dim3 mm_grid(int M, int N, int S) {
    return dim3((unsigned)((M + MM_T - 1) / MM_T), (unsigned)((N + MM_T - 1) / MM_T), (unsigned)S);
}

// One product op(P) op(Q) (MmArgs fields filled by the caller) over the whole k.
template <bool TP, bool TQ, int EPI>
static void mm(MmArgs a, hipStream_t s) {
    a.kchunk = a.K > 0 ? a.K : 1;
    hipLaunchKernelGGL((mm_kernel<TP, TQ, EPI>), mm_grid(a.M, a.N, 1), dim3(256), 0, s, a);
}

// k ranges of a gradient product over `rows` training rows: about 512 blocks in
// all, at least 64 rows per range (multiples of MM_K).
struct GradSplit {
    int S;
    int64_t kchunk;
};

static GradSplit grad_split(int M, int N1, int64_t rows) {
    const int64_t tiles = (int64_t)((M + MM_T - 1) / MM_T) * ((N1 + MM_T - 1) / MM_T);
    int64_t want = 512 / tiles > 1 ? 512 / tiles : 1;
    int64_t kc = (rows + want - 1) / want;
    if (kc < 64) kc = 64;
    kc = (kc + MM_K - 1) / MM_K * MM_K;
    return {(int)((rows + kc - 1) / kc), kc};
}

// Elements of the partial-plane buffer a training set of `rows` rows needs.
static int64_t planes_elems(const Mlp *p, int64_t rows) {
    const int dims[3][2] = {{p->O, p->H + 1}, {p->H, p->H + 1}, {p->H, p->I + 1}};
    int64_t most = 0;
    for (auto &d : dims) {
        const GradSplit g = grad_split(d[0], d[1], rows);
        most = std::max<int64_t>(most, (int64_t)g.S * d[0] * d[1]);
    }
    return most;
}

// gW (M x N) and gb (M) = dZ^T [A | 1] over the B rows: dZ is B x M (ld M), A is
// B x N (ld N); scale: the factor of dZ (NULL: 1).
static void grad_product(Mlp *p, const float *dZ, int M, const float *A, int N,
                         const float *scale, float *gW, float *gb, hipStream_t s) {
    const GradSplit g = grad_split(M, N + 1, p->B);
    MmArgs a = {};
    a.P = dZ;
    a.ldp = M;
    a.Q = A;
    a.ldq = N;
    a.M = M;
    a.N = N + 1;
    a.K = p->B;
    a.kchunk = g.kchunk;
    a.ones_col = N;
    a.scale = scale;
    a.C = p->planes;
    a.ldc = N + 1;
    a.plane = (int64_t)M * (N + 1);
    hipLaunchKernelGGL((mm_kernel<true, false, MM_PARTIAL>), mm_grid(M, N + 1, g.S), dim3(256), 0, s,
                       a);
    hipLaunchKernelGGL(mm_reduce_kernel, dim3(nblk(a.plane)), dim3(256), 0, s, p->planes, g.S, M, N,
                       gW, gb);
}

// Forward pass of B rows: h1, h2 (and z1, z2 when given) and y.  With T and D the
// output layer also forms D = M (y - T) and its per-tile loss sums in p->part.
static void mlp_forward_launch(Mlp *p, int64_t B, const float *X, float *z1, float *h1, float *z2,
                               float *h2, float *y, const float *T, const float *Mk, float *D,
                               hipStream_t s) {
    MmArgs a = {};
    a.ones_col = -1;
    a.M = (int)B;
    // layer 1: z1 = X W1^T + b1
    a.P = X; a.ldp = p->I; a.Q = p->W1(); a.ldq = p->I; a.N = p->H; a.K = p->I;
    a.bias = p->b1(); a.C = h1; a.ldc = p->H; a.Z2 = z1;
    mm<false, true, MM_BIAS_RELU>(a, s);
    // layer 2: z2 = h1 W2^T + b2
    a.P = h1; a.ldp = p->H; a.Q = p->W2(); a.ldq = p->H; a.N = p->H; a.K = p->H;
    a.bias = p->b2(); a.C = h2; a.ldc = p->H; a.Z2 = z2;
    mm<false, true, MM_BIAS_RELU>(a, s);
    // output layer: y = h2 W3^T + b3
    a.P = h2; a.ldp = p->H; a.Q = p->W3(); a.ldq = p->H; a.N = p->O; a.K = p->H;
    a.bias = p->b3(); a.C = y; a.ldc = p->O; a.Z2 = nullptr;
    if (D) {
        a.T = T; a.Mk = Mk; a.Z2 = D; a.part = p->part;
        mm<false, true, MM_BIAS_LOSS>(a, s);
    } else {
        mm<false, true, MM_BIAS>(a, s);
    }
}

// forward + loss + backward on the training set (gradients into p->grad)
static void mlp_grad_launch(Mlp *p, hipStream_t s, bool count_step) {
    const int64_t B = p->B;
    const int I = p->I, H = p->H, O = p->O;
    mlp_forward_launch(p, B, p->X, p->z1, p->h1, p->z2, p->h2, p->y, p->T, p->M, p->d, s);
    const dim3 g3 = mm_grid((int)B, O, 1);
    hipLaunchKernelGGL(mlp_loss_final_kernel, dim3(1), dim3(256), 0, s, p->part,
                       (int)(g3.x * g3.y), p->loss, p->loss + 1,
                       count_step ? p->step : (int *)nullptr);
    const float *scale = p->loss + 1;      // dL/dy = scale * d
    grad_product(p, p->d, O, p->h2, H, scale, p->gW3(), p->gb3(), s);
    MmArgs a = {};
    a.ones_col = -1;
    a.M = (int)B;
    // dz2 = (dL/dy W3) * (z2 > 0)
    a.P = p->d; a.ldp = O; a.Q = p->W3(); a.ldq = H; a.N = H; a.K = O;
    a.scale = scale; a.Zp = p->z2; a.C = p->dz2; a.ldc = H;
    mm<false, false, MM_MASK>(a, s);
    grad_product(p, p->dz2, H, p->h1, H, nullptr, p->gW2(), p->gb2(), s);
    // dz1 = (dz2 W2) * (z1 > 0)
    a.P = p->dz2; a.ldp = H; a.Q = p->W2(); a.ldq = H; a.N = H; a.K = H;
    a.scale = nullptr; a.Zp = p->z1; a.C = p->dz1; a.ldc = H;
    mm<false, false, MM_MASK>(a, s);
    grad_product(p, p->dz1, H, p->X, I, nullptr, p->gW1(), p->gb1(), s);
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
    if (rows < 1 || rows > MLP_MAX_ROWS) return set_error(-2, "rows outside [1, 2^30]");
    if (!X) return set_error(-3, "X is NULL");
    if (!T) return set_error(-4, "T is NULL");
    if (!M) return set_error(-5, "M is NULL");
    hipError_t se = hipStreamSynchronize(current_stream());
    if (se != hipSuccess) return hip_err(se, "mlp_set_data");
    free_data(p);
    const int64_t B = rows;
    const int64_t tiles3 = ((B + MM_T - 1) / MM_T) * ((p->O + MM_T - 1) / MM_T);
    p->B = B;    // for planes_elems; reset below on failure
    struct { float **dst; int64_t n; } bufs[] = {
        {&p->X, B * p->I}, {&p->T, B * p->O}, {&p->M, B * p->O}, {&p->z1, B * p->H},
        {&p->h1, B * p->H}, {&p->z2, B * p->H}, {&p->h2, B * p->H}, {&p->y, B * p->O},
        {&p->d, B * p->O}, {&p->dz2, B * p->H}, {&p->dz1, B * p->H},
        {&p->planes, planes_elems(p, B)}, {&p->part, 2 * tiles3}};
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
    if (rows < 0 || rows > MLP_MAX_ROWS) return set_error(-2, "rows outside [0, 2^30]");
    if (rows == 0) return 0;
    if (!X) return set_error(-3, "X is NULL");
    if (!Y) return set_error(-4, "Y is NULL");
    float *tmp = nullptr;
    const int64_t B = rows;
    hipError_t e = hipMalloc((void **)&tmp, (size_t)B * p->H * 2 * sizeof(float));
    if (e != hipSuccess) return set_error(MGEMM_ERR_NOMEM, "mlp_forward: scratch");
    hipStream_t s = current_stream();
    mlp_forward_launch(p, B, X, (float *)nullptr, tmp, (float *)nullptr, tmp + B * p->H, Y,
                       (const float *)nullptr, (const float *)nullptr, (float *)nullptr, s);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    return e == hipSuccess ? 0 : hip_err(e, "mlp_forward");
}

int32_t mlp_predict(void *handle, int64_t rows, const float *X, const float *M, int32_t *idx) {
    Mlp *p = (Mlp *)handle;
    if (!p) return set_error(-1, "handle is NULL");
    if (rows < 0 || rows > MLP_MAX_ROWS) return set_error(-2, "rows outside [0, 2^30]");
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
