// The learned tile-configuration model behind the C ABI: a trained 3-layer MLP
// (mlp.hip) with its feature scaling and the configuration each output stands
// for, saved to and loaded from a text file, and evaluated by the library's own
// HIP kernels to choose a configuration for an unseen shape.
//
// The paper fixes its tuning parameters per architecture from exhaustive search
// (Sec. 3, Tab. 4) and names tuning itself as the task that grows with the
// number of parameters (Sec. 6); the model replaces the search for a new shape
// by one evaluation of the network.
//
// File format (ASCII lines; every floating-point value as a C99 hexadecimal
// float, so that it is read back exactly):
//   mgemm-mlp 2
//   dims <in> <hidden> <out>
//   out <dtype> <bm> <bn> <bk> <waves> <elems_per_thread> <double_buffer> <occupancy>
//       (one line per output, in output order)
//   mean <in values>                 feature means (double)
//   std <in values>                  feature standard deviations (double, > 0)
//   params <count>
//   <count values, 8 per line>       W1 b1 W2 b2 W3 b3 (float), row-major
//   checksum <16 hex digits>         FNV-1a (64-bit) of every byte before this line
// Features of an m x n x k product of dtype d: x = [log2 m, log2 n, log2 k,
// d == F64, d == F32, w], w = 1 where the rows of A and B are whole 16-byte loads
// (n, lda and ldb multiples of 2 in FP64, of 4 in FP32, A and B 16-byte aligned:
// the three-stage kernels run only then), scaled as (x - mean) / std in double and
// rounded to float.  The prediction is the output with the largest value among
// those whose dtype is d (lowest index on ties).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mgemm_internal.h"

namespace mgemm {

int32_t set_error(int32_t code, const char *fmt, ...);
hipStream_t current_stream();
bool cfg_registered(int32_t dtype, const mgemm_cfg &c);

constexpr int MODEL_IN = 6;
constexpr int MODEL_MAX_DIM = 4096;
constexpr int MODEL_MAX_DEVICES = 64;

static uint64_t fnv1a(const char *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= (uint8_t)p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

static void put(std::string &s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static void put(std::string &s, const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    const int n = vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n > 0) s.append(buf, (size_t)std::min(n, (int)sizeof buf - 1));
}

int32_t model_write(const char *path, int I, int H, int O, const int32_t *out_dtype,
                    const mgemm_cfg *out_cfg, const double *mean, const double *stdv,
                    const float *params, int64_t P) {
    std::string s;
    put(s, "mgemm-mlp 2\ndims %d %d %d\n", I, H, O);
    for (int o = 0; o < O; ++o) {
        const mgemm_cfg &c = out_cfg[o];
        put(s, "out %d %d %d %d %d %d %d %d\n", (int)out_dtype[o], (int)c.bm, (int)c.bn, (int)c.bk,
            (int)c.waves, (int)c.elems_per_thread, (int)c.double_buffer, (int)c.occupancy);
    }
    s += "mean";
    for (int i = 0; i < I; ++i) put(s, " %a", mean[i]);
    s += "\nstd";
    for (int i = 0; i < I; ++i) put(s, " %a", stdv[i]);
    put(s, "\nparams %lld\n", (long long)P);
    for (int64_t i = 0; i < P; ++i) put(s, "%a%c", (double)params[i], (i % 8 == 7 || i + 1 == P) ? '\n' : ' ');
    put(s, "checksum %016llx\n", (unsigned long long)fnv1a(s.data(), s.size()));
    FILE *f = fopen(path, "wb");
    if (!f) return set_error(MGEMM_ERR_MODEL, "model: cannot write %s", path);
    const size_t w = fwrite(s.data(), 1, s.size(), f);
    const int cl = fclose(f);
    if (w != s.size() || cl != 0) return set_error(MGEMM_ERR_MODEL, "model: short write to %s", path);
    return 0;
}

struct Model {
    int I = 0, H = 0, O = 0;
    std::vector<int32_t> out_dtype;
    std::vector<mgemm_cfg> out_cfg;
    std::vector<double> mean, stdv;
    std::vector<float> params;
    // per device: the network and its one-row input, mask and result buffers
    void *net[MODEL_MAX_DEVICES] = {};
    float *dx[MODEL_MAX_DEVICES] = {};
    float *dm[MODEL_MAX_DEVICES] = {};
    int32_t *didx[MODEL_MAX_DEVICES] = {};
    std::map<std::tuple<int32_t, int64_t, int64_t, int64_t, bool>, int> cache;
};

static std::mutex g_model_mtx;
static Model *g_model = nullptr;

// Parses and checks a model file's text; returns 0 and fills *out, or an error.
static int32_t model_parse(const std::string &text, const char *path, Model *out) {
    const size_t cpos = text.rfind("checksum ");
    if (cpos == std::string::npos || (cpos > 0 && text[cpos - 1] != '\n'))
        return set_error(MGEMM_ERR_MODEL, "model %s: no checksum line", path);
    unsigned long long want = 0;
    if (sscanf(text.c_str() + cpos, "checksum %16llx", &want) != 1)
        return set_error(MGEMM_ERR_MODEL, "model %s: unreadable checksum", path);
    if (fnv1a(text.data(), cpos) != want)
        return set_error(MGEMM_ERR_MODEL, "model %s: checksum mismatch (corrupt file)", path);
    const std::string body = text.substr(0, cpos);
    const char *p = body.c_str();
    char *end = nullptr;
    auto word = [&](const char *w) {
        while (*p == ' ' || *p == '\n') ++p;
        const size_t n = strlen(w);
        if (strncmp(p, w, n) != 0 || (p[n] != ' ' && p[n] != '\n')) return false;
        p += n;
        return true;
    };
    auto integer = [&](long long *v) {
        *v = strtoll(p, &end, 10);
        if (end == p) return false;
        p = end;
        return true;
    };
    auto real = [&](double *v) {
        *v = strtod(p, &end);
        if (end == p) return false;
        p = end;
        return true;
    };
    long long ver = 0, I = 0, H = 0, O = 0;
    if (!word("mgemm-mlp") || !integer(&ver) || ver != 2)
        return set_error(MGEMM_ERR_MODEL, "model %s: not an mgemm-mlp version 2 file", path);
    if (!word("dims") || !integer(&I) || !integer(&H) || !integer(&O))
        return set_error(MGEMM_ERR_MODEL, "model %s: bad dims line", path);
    if (I != MODEL_IN)
        return set_error(MGEMM_ERR_MODEL, "model %s: %lld inputs, the features are %d", path, I,
                         MODEL_IN);
    if (H < 1 || H > MODEL_MAX_DIM || O < 1 || O > MODEL_MAX_DIM)
        return set_error(MGEMM_ERR_MODEL, "model %s: dims outside 1..%d", path, MODEL_MAX_DIM);
    out->I = (int)I;
    out->H = (int)H;
    out->O = (int)O;
    for (long long o = 0; o < O; ++o) {
        long long v[8];
        if (!word("out"))
            return set_error(MGEMM_ERR_MODEL, "model %s: output %lld missing", path, o);
        for (long long &x : v)
            if (!integer(&x))
                return set_error(MGEMM_ERR_MODEL, "model %s: output %lld unreadable", path, o);
        const mgemm_cfg c = {(int32_t)v[1], (int32_t)v[2], (int32_t)v[3], (int32_t)v[4],
                             (int32_t)v[5], (int32_t)v[6], (int32_t)v[7]};
        if ((v[0] != MGEMM_F64 && v[0] != MGEMM_F32) || !cfg_registered((int32_t)v[0], c))
            return set_error(MGEMM_ERR_MODEL,
                             "model %s: output %lld names dtype %lld configuration "
                             "%dx%dx%d w%d e%d d%d o%d, which this library does not register",
                             path, o, v[0], c.bm, c.bn, c.bk, c.waves, c.elems_per_thread,
                             c.double_buffer, c.occupancy);
        out->out_dtype.push_back((int32_t)v[0]);
        out->out_cfg.push_back(c);
    }
    for (const char *name : {"mean", "std"}) {
        std::vector<double> &dst = name[0] == 'm' ? out->mean : out->stdv;
        if (!word(name)) return set_error(MGEMM_ERR_MODEL, "model %s: no %s line", path, name);
        for (long long i = 0; i < I; ++i) {
            double x;
            if (!real(&x) || !isfinite(x) || (name[0] == 's' && !(x > 0.0)))
                return set_error(MGEMM_ERR_MODEL, "model %s: bad %s value", path, name);
            dst.push_back(x);
        }
    }
    long long P = 0;
    const long long want_p = H * I + H + H * H + H + O * H + O;
    if (!word("params") || !integer(&P) || P != want_p)
        return set_error(MGEMM_ERR_MODEL, "model %s: parameter count is not %lld", path, want_p);
    out->params.reserve((size_t)P);
    for (long long i = 0; i < P; ++i) {
        double x;
        if (!real(&x) || !isfinite(x) || (float)x != x)
            return set_error(MGEMM_ERR_MODEL, "model %s: parameter %lld unreadable", path, i);
        out->params.push_back((float)x);
    }
    while (*p == ' ' || *p == '\n') ++p;
    if (*p) return set_error(MGEMM_ERR_MODEL, "model %s: trailing text before the checksum", path);
    return 0;
}

static void model_free(Model *md) {
    if (!md) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < MODEL_MAX_DEVICES; ++d) {
        if (!md->net[d] && !md->dx[d]) continue;
        // teardown: nothing more can be done about a failure here
        (void)hipSetDevice(d);
        if (md->net[d]) (void)mlp_destroy(md->net[d]);
        if (md->dx[d]) (void)hipFree(md->dx[d]);
        if (md->dm[d]) (void)hipFree(md->dm[d]);
        if (md->didx[d]) (void)hipFree(md->didx[d]);
    }
    if (have) (void)hipSetDevice(cur);
    delete md;
}

// The model's choice for a shape (caller holds g_model_mtx).  may_launch false:
// only a cached choice is returned (MGEMM_ERR_MODEL otherwise, without text).
static int32_t model_choose_locked(int32_t dtype, int64_t m, int64_t n, int64_t k, bool rows16,
                                   bool may_launch, mgemm_cfg *out) {
    Model *md = g_model;
    const auto key = std::make_tuple(dtype, m, n, k, rows16);
    auto it = md->cache.find(key);
    if (it != md->cache.end()) {
        *out = md->out_cfg[it->second];
        return 0;
    }
    if (!may_launch) return MGEMM_ERR_MODEL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MODEL_MAX_DEVICES)
        return set_error(MGEMM_ERR_HIP, "model: no usable current device");
    if (!md->net[dev]) {
        int32_t rc = mlp_create(md->I, md->H, md->O, md->params.data(), &md->net[dev]);
        if (rc) return rc;
        e = hipMalloc((void **)&md->dx[dev], sizeof(float) * md->I);
        if (e == hipSuccess) e = hipMalloc((void **)&md->dm[dev], sizeof(float) * md->O);
        if (e == hipSuccess) e = hipMalloc((void **)&md->didx[dev], sizeof(int32_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(MGEMM_ERR_NOMEM, "model: device buffers");
        }
    }
    const double raw[MODEL_IN] = {log2((double)m), log2((double)n), log2((double)k),
                                  dtype == MGEMM_F64 ? 1.0 : 0.0, dtype == MGEMM_F32 ? 1.0 : 0.0,
                                  rows16 ? 1.0 : 0.0};
    float x[MODEL_IN];
    for (int i = 0; i < MODEL_IN; ++i) x[i] = (float)((raw[i] - md->mean[i]) / md->stdv[i]);
    std::vector<float> mask((size_t)md->O);
    for (int o = 0; o < md->O; ++o) mask[o] = md->out_dtype[o] == dtype ? 1.0f : 0.0f;
    e = hipMemcpy(md->dx[dev], x, sizeof x, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(md->dm[dev], mask.data(), sizeof(float) * md->O, hipMemcpyHostToDevice);
    if (e != hipSuccess) return set_error(MGEMM_ERR_HIP, "model: %s", hipGetErrorString(e));
    int32_t rc = mlp_predict(md->net[dev], 1, md->dx[dev], md->dm[dev], md->didx[dev]);
    if (rc) return rc;
    int32_t idx = -1;
    e = hipMemcpy(&idx, md->didx[dev], sizeof idx, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_error(MGEMM_ERR_HIP, "model: %s", hipGetErrorString(e));
    if (idx < 0 || idx >= md->O) return set_error(MGEMM_ERR_MODEL, "model: no output for dtype %d", dtype);
    md->cache[key] = idx;
    *out = md->out_cfg[idx];
    return 0;
}

// gemm_ex's use of a loaded model: 0 with *out set, or nonzero (no model, no
// cached choice when may_launch is false, or a failed evaluation) -- the caller
// then keeps the built-in choice.
int32_t model_choose(int32_t dtype, int64_t m, int64_t n, int64_t k, bool rows16, bool may_launch,
                     mgemm_cfg *out) {
    std::lock_guard<std::mutex> lock(g_model_mtx);
    if (!g_model) return MGEMM_ERR_MODEL;
    for (int o = 0; o < g_model->O; ++o)
        if (g_model->out_dtype[o] == dtype)
            return model_choose_locked(dtype, m, n, k, rows16, may_launch, out);
    return MGEMM_ERR_MODEL;
}

}  // namespace mgemm

using namespace mgemm;

extern "C" {

int32_t mgemm_model_load(const char *path) {
    Model *md = nullptr;
    if (path) {
        FILE *f = fopen(path, "rb");
        if (!f) return set_error(MGEMM_ERR_MODEL, "model: cannot open %s", path);
        std::string text;
        char buf[65536];
        size_t r;
        while ((r = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
        const bool bad = ferror(f) != 0;
        fclose(f);
        if (bad) return set_error(MGEMM_ERR_MODEL, "model: read error on %s", path);
        md = new Model();
        const int32_t rc = model_parse(text, path, md);
        if (rc) {
            delete md;
            return rc;
        }
    }
    Model *old = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_model_mtx);
        old = g_model;
        g_model = md;
    }
    model_free(old);
    return 0;
}

int32_t mgemm_model_predict(int64_t m, int64_t n, int64_t k, int32_t dtype, mgemm_cfg *out) {
    if (m < 1) return set_error(-1, "m < 1");
    if (n < 1) return set_error(-2, "n < 1");
    if (k < 1) return set_error(-3, "k < 1");
    if (!out) return set_error(-5, "out is NULL");
    std::lock_guard<std::mutex> lock(g_model_mtx);
    if (!g_model) return set_error(MGEMM_ERR_MODEL, "no model loaded");
    bool has = false;
    for (int o = 0; o < g_model->O && !has; ++o) has = g_model->out_dtype[o] == dtype;
    if (!has) return set_error(-4, "the loaded model has no output for dtype %d", dtype);
    // rows of a product stored without padding (lda = k, ldb = n)
    const int64_t epu = dtype == MGEMM_F32 ? 4 : 2;
    return model_choose_locked(dtype, m, n, k, n % epu == 0 && k % epu == 0, true, out);
}

}  // extern "C"
