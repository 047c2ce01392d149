/*
 * mgemm -- tiled general matrix multiply C = alpha*A*B + beta*C on AMD MI355X
 * (gfx950), behind a plain C ABI.
 *
 * The operation is the paper's benchmark computation (Matthes et al., "Tuning and
 * optimization for a variety of many-core architectures without changing a single
 * line of implementation code using the Alpaka library", Sec. 2, Eq. 1): square in
 * the paper, general m x n x k here.  Its work is counted as 2*m*n*k floating-point
 * operations (Sec. 2, Eq. 2 and Eq. 4 keep the leading 2N^3 term).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout   Row-major.  A is m x k with lda >= max(1,k); B is k x n with
 *          ldb >= max(1,n); C is m x n with ldc >= max(1,n).  Leading dimensions
 *          count elements.  There are no transpose flags (the paper has none).
 * Pointers A, B, C are DEVICE pointers on the current HIP device (device memory,
 *          or the device address of mapped host memory, mgemm_host_alloc).  The caller owns
 *          them; the library never frees, reallocates or keeps them after the call
 *          (batched plans keep them until destroyed, see below).  C must not
 *          overlap A or B.
 * Types    MGEMM_F64: A, B, C are double.  MGEMM_F32: float (alpha, beta are
 *          rounded to float).  MGEMM_SPLIT_BF16 / MGEMM_SPLIT_FP8 /
 *          MGEMM_SPLIT_INT8: A, B, C are double; the product is emulated from
 *          bfloat16 (6 slices, 21 slice pairs) / FP8 e4m3 (11 slices, 66 pairs) /
 *          int8 (8 slices, 36 pairs) slices of A and B (Ozaki scheme), see
 *          gemm_ex.  MGEMM_CRT_INT8: A, B, C are double; the product
 *          is emulated from int8 residues of A and B modulo 16 coprime moduli
 *          (Ozaki scheme II), see gemm_ex.
 * Stream   Work is enqueued on the given HIP stream (NULL: the stream set with
 *          mgemm_set_stream, by default the null stream) and the call returns
 *          after enqueueing.  Launch errors are reported at once; faults surface
 *          at the caller's synchronisation.
 * Quick    m == 0 or n == 0: nothing happens.  k == 0 or alpha == 0: C = beta*C
 * returns  and A, B are not read.  beta == 0: C is written without being read (a
 *          NaN already in C does not propagate).  Padding columns (ldc > n) are
 *          never written.
 * Errors   0 on success.  -i: argument i (1-based, BLAS "info" convention) is
 *          invalid, e.g. -1 for m < 0, -6 for lda < max(1,k), -12 for an unknown
 *          dtype, or a NULL pointer whose matrix is non-empty.  Positive codes are
 *          run-time errors: MGEMM_ERR_HIP (text in mgemm_last_error()),
 *          MGEMM_ERR_NOMEM, MGEMM_ERR_NONFINITE (split paths: NaN or Inf in A or
 *          B), MGEMM_ERR_NOCONFIG, MGEMM_ERR_PLAN, MGEMM_ERR_MODEL (a cost-model
 *          file that cannot be read, is corrupt or does not match the library, or
 *          no model loaded).  On any error C is untouched.
 * Threads  Calls may come from several host threads; the error text is
 *          per thread.  Concurrent calls that share a split-path workspace on
 *          one device are serialised by the library.
 */
#ifndef MGEMM_H
#define MGEMM_H

#include <stdint.h>

#define MGEMM_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MGEMM_F64 = 0,
    MGEMM_F32 = 1,
    MGEMM_SPLIT_BF16 = 2,
    MGEMM_SPLIT_FP8 = 3,
    MGEMM_SPLIT_INT8 = 4,
    MGEMM_CRT_INT8 = 5
} mgemm_dtype;

enum {
    MGEMM_OK = 0,
    MGEMM_ERR_HIP = 1,
    MGEMM_ERR_NOMEM = 2,
    MGEMM_ERR_NONFINITE = 3,
    MGEMM_ERR_NOCONFIG = 4,
    MGEMM_ERR_PLAN = 5,
    MGEMM_ERR_MODEL = 6
};

/*
 * A tile configuration (the paper's tuning parameters, Sec. 2.1 Listing 1 and
 * Sec. 3 Tab. 4: tile size T and elements per thread, generalised).
 *   bm, bn, bk        work-group tile of C (bm x bn) and depth of one k-step.
 *   waves             64-lane wavefronts per work-group.
 *   elems_per_thread  contiguous elements one thread copies per global->LDS
 *                     load (the paper's element layer).
 *   double_buffer     1: two LDS stages, the next k-step's tiles are loaded while
 *                     the current one is multiplied; 0: one stage; 2: three
 *                     stages filled by direct global->LDS loads two k-steps
 *                     ahead (needs n, lda and ldb multiples of the 16-byte load,
 *                     2 FP64 or 4 FP32 elements, and 16-byte aligned A and B,
 *                     else the two-stage kernel of the same tile runs, with the
 *                     same results).
 *   occupancy         wavefronts per SIMD the kernel is compiled to allow (0: the
 *                     compiler's choice, else 1 or 2) -- the GPU counterpart of
 *                     the paper's hardware threads per core (Sec. 3, Tab. 4).
 */
typedef struct {
    int32_t bm, bn, bk, waves, elems_per_thread, double_buffer, occupancy;
} mgemm_cfg;

/* C = alpha*A*B + beta*C (Eq. 1) with the library's choice of tile configuration,
 * on the library's current stream.  Arguments are numbered 1..12 as written. */
MGEMM_API int32_t gemm(int64_t m, int64_t n, int64_t k, double alpha,
             const void *A, int64_t lda, const void *B, int64_t ldb,
             double beta, void *C, int64_t ldc, int32_t dtype);

/* gemm with an explicit configuration (cfg == NULL: the library's choice; a cfg
 * that is not in the registry for dtype gives -13) and stream (argument 14,
 * a hipStream_t; NULL: the current library stream).
 *
 * The library's choice (MGEMM_F64, MGEMM_F32): the largest preferred tile that
 * still gives enough work-groups for the m x n output; split-k below where k >=
 * 2048 or m, n or k lies outside [64, 16384]; otherwise, with a cost model loaded
 * (mgemm_model_load) and m, n, k in [64, 16384], its prediction; else, for rows
 * the three-stage kernels can load (n, lda, ldb multiples of 16 bytes, A and B
 * 16-byte aligned), the three-stage tile (256 x 128, 128 x 128 or 64 x 64) whose
 * sustained rate times the fill of its rounds of one work-group per compute unit
 * is highest, if that fill is at least 80 % -- or, where 128 x 128 tiles leave a
 * last round of few tiles, the tile rows that fill whole rounds whole and the
 * remaining rows with k cut (a split tail), where that is estimated 5 % faster
 * than the best single tile (2 % where that tile is 128 x 128 or 256 x 128);
 * else (m, n, k in [64, 16384]), for
 * rows the three-stage kernels cannot load or where the preferred tile is a
 * two-stage one, the configuration measured fastest on the tuner's shapes of the
 * same row class in and around the (floor(log2 m), floor(log2 n), floor(log2 k))
 * cell.
 *
 * Split-k (MGEMM_F64 and MGEMM_F32, cfg == NULL only, k >= 2048 or outside the
 * measured range): when the preferred tile leaves fewer than about four
 * work-groups per compute unit and k >= 512, k is
 * cut into S <= 16 ranges (multiples of 256; computed with the three-stage
 * 128 x 128 tile where its requirements hold and it fills the GPU, else, for
 * MGEMM_F64 only, with the chosen tile); their partial products go to the library-owned
 * device workspace (S*m*n*8 bytes, S*m*n*4 for FP32, grown on demand, MGEMM_ERR_NOMEM if it
 * cannot be, kept until mgemm_release_workspace(); calls on one device that use
 * it are ordered through it) and one kernel adds them in range order and applies
 * alpha and beta.  Results are deterministic; they can differ in the last bits
 * from the same tile run with an explicit cfg (another summation order).
 *
 * Split dtypes: A and B are scaled per row / column by powers of two, sliced
 * into small integers and multiplied on matrix cores with exact accumulation;
 * the kept slice-pair products (s + t <= S + 1) are summed exactly and rounded
 * once to FP64, then C = alpha*v + beta*C.  For k above 131072 (bf16, FP8) or
 * 16384 (int8) the k-range is processed in passes, each rounded once.  The slices
 * live in a library-owned device workspace (about 2*S*bytes*(m+n)*k, plus 16
 * bytes per element of C for FP8) that grows on demand (MGEMM_ERR_NOMEM if it
 * cannot; MGEMM_ERR_NOCONFIG if the int8 or FP8 slices of one operand pass 4 GiB)
 * and is kept until
 * mgemm_release_workspace() or unload.  The call waits once for the scaling
 * step on the stream (to report MGEMM_ERR_NONFINITE before C is touched);
 * split calls on one device are ordered through the shared workspace. cfg must
 * be NULL.
 *
 * MGEMM_CRT_INT8 (modular-integer emulation, Ozaki scheme II): with e_i, f_j the
 * exponents of the row maxima of A and column maxima of B and b the largest
 * integer <= 62 with k 2^(2b) <= 2^123, the operands are truncated to integers
 * A'_ip = trunc(A_ip 2^(b-e_i)), B'_pj = trunc(B_pj 2^(b-f_j)) (|.| < 2^b); the
 * exact C'_ij = sum_p A'_ip B'_pj is obtained from 16 int8 GEMMs of their
 * residues modulo 16 pairwise coprime moduli (Chinese remainder theorem), rounded
 * once to FP64, scaled by 2^(e_i+f_j-2b), and C = alpha*v + beta*C.  k is limited
 * to 2^24 - 64 (MGEMM_ERR_NOCONFIG above); the workspace (same rules as above)
 * holds about 16*((m+n)*k + m*n) bytes.  Non-finite input: MGEMM_ERR_NONFINITE, C
 * untouched.  cfg must be NULL. */
MGEMM_API int32_t gemm_ex(int64_t m, int64_t n, int64_t k, double alpha,
                const void *A, int64_t lda, const void *B, int64_t ldb,
                double beta, void *C, int64_t ldc, int32_t dtype,
                const mgemm_cfg *cfg, void *stream);

/* gemm_ex without device allocation, for callers that cannot allocate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, checks, choice and results as gemm_ex (bitwise, for the same
 * configuration and split of k) for dtype MGEMM_F64 and MGEMM_F32; any other
 * dtype returns -12 (the emulated dtypes need the library workspace).  A loaded
 * cost model (mgemm_model_load) is used only for shapes whose choice it has
 * already cached (it is never evaluated here); otherwise the built-in choice
 * applies.  The split-k partial products go to a 64 MiB device array of the
 * library (one per GPU, kept until the process ends), which every split-k plan
 * of a 256-CU GPU fits; a plan that would need more returns MGEMM_ERR_NOMEM
 * with the sizes in mgemm_last_error().  Every call on one GPU shares that
 * array: calls that overlap on one GPU (different streams, several threads)
 * race; order them on one stream.  Asynchronous on the stream like gemm_ex. */
MGEMM_API int32_t gemm_ex_noalloc(int64_t m, int64_t n, int64_t k, double alpha,
                                  const void *A, int64_t lda, const void *B, int64_t ldb,
                                  double beta, void *C, int64_t ldc, int32_t dtype,
                                  const mgemm_cfg *cfg, void *stream);

/*
 * Batched GEMM: count independent problems C_i = alpha_i A_i B_i + beta_i C_i
 * (Eq. 1 per problem), dtype MGEMM_F64 or MGEMM_F32 for plans (any dtype for
 * gemm_batched).  All array arguments are HOST arrays of count entries; A, B, C
 * hold DEVICE pointers.  Problem arguments are checked as in gemm (an invalid
 * problem returns that argument's -i code and names the problem in
 * mgemm_last_error).
 *
 * gemm_batched: one gemm launch per problem, in order, on the current stream.
 * Array arguments are numbered 2..12 after count (1); dtype is 13.
 */
MGEMM_API int32_t gemm_batched(int64_t count, const int64_t *m, const int64_t *n,
                               const int64_t *k, const double *alpha, const void *const *A,
                               const int64_t *lda, const void *const *B, const int64_t *ldb,
                               const double *beta, void *const *C, const int64_t *ldc,
                               int32_t dtype);

/* Builds a reusable plan for one batched launch: problems are grouped by tile
 * configuration (cfgs[i], argument 14: a registered configuration with the
 * MGEMM_CFG_BATCHED flag, else -14; when cfgs is NULL every problem uses the
 * registered 64x64x16 four-wave configuration); per group one persistent kernel takes C
 * tiles from per-XCD atomic work lists, each tile running the code path of its
 * problem's row alignment; all groups are captured into one HIP graph.  The plan keeps the problem
 * descriptors (pointers, sizes, alpha, beta) -- the matrices must stay valid and
 * are read at each execution.  Problems with k == 0 or alpha == 0 are rejected
 * (MGEMM_ERR_PLAN).  stream: the stream executions run on (NULL: null stream).
 * Results are bitwise identical to gemm_ex with the same configurations.
 * *plan receives an opaque handle; returns 0 or an error code. */
MGEMM_API int32_t gemm_batched_plan_create(int64_t count, const int64_t *m, const int64_t *n,
                                           const int64_t *k, const double *alpha,
                                           const void *const *A, const int64_t *lda,
                                           const void *const *B, const int64_t *ldb,
                                           const double *beta, void *const *C,
                                           const int64_t *ldc, int32_t dtype,
                                           const mgemm_cfg *cfgs, void *stream, void **plan);

/* Runs a plan: one hipGraphLaunch on the plan's stream (asynchronous).
 * Executions of one plan must not overlap (they share the work counters). */
MGEMM_API int32_t gemm_batched_plan_execute(void *plan);

/* Waits for the plan's stream and frees the plan (NULL is a no-op); returns
 * MGEMM_ERR_HIP if that wait reported an error (the plan is freed anyway). */
MGEMM_API int32_t gemm_batched_plan_destroy(void *plan);

/* Number of configuration groups, total C tiles and total 2*m*n*k of a plan. */
MGEMM_API int32_t gemm_batched_plan_info(void *plan, int32_t *buckets, int64_t *total_tiles,
                                         double *flops);

/*
 * The learned tile-configuration cost model: a 3-layer FP32 MLP
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3
 * trained with the masked mean square loss sum M (y - t)^2 / sum M and Adam
 * (Kingma and Ba, ICLR 2015), entirely by the library's HIP kernels.  The paper
 * hopes its tuning parameters enable automatic tuning (Sec. 1.1) and finds that
 * tuning itself becomes a compute-intensive task as parameters are added
 * (Sec. 6); the model predicts a configuration instead of measuring all.
 *
 * Parameters are one flat FP32 vector W1 (hidden x in), b1, W2 (hidden x hidden),
 * b2, W3 (out x hidden), b3, row-major.  Host arrays are marked (host), the rest
 * are device pointers.  All calls run on the library's current stream and return
 * after it has finished.  Dimensions are limited to 1..4096.
 */
/* Creates a model with the given initial parameters (host, mlp_param_count
 * floats); Adam moments start at zero.  *mlp receives the handle. */
MGEMM_API int32_t mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim,
                             const float *init_params, void **mlp);
/* Number of parameters (-1 for a NULL handle). */
MGEMM_API int64_t mlp_param_count(void *mlp);
/* Copies the parameters in (host) and resets the Adam state. */
MGEMM_API int32_t mlp_set_params(void *mlp, const float *params);
/* Copies the parameters out (host). */
MGEMM_API int32_t mlp_get_params(void *mlp, float *params);
/* Sets the training set: X rows x in, targets T and mask M rows x out (device;
 * copied into library buffers). */
MGEMM_API int32_t mlp_set_data(void *mlp, int64_t rows, const float *X, const float *T,
                               const float *M);
/* Loss and gradient (host outputs, either may be NULL) on the training set,
 * without an update. */
MGEMM_API int32_t mlp_loss_grad(void *mlp, float *loss, float *grad);
/* steps full-batch Adam steps (one captured HIP graph per step); *last_loss
 * (host, may be NULL) receives the loss evaluated in the last step. */
MGEMM_API int32_t mlp_train(void *mlp, int32_t steps, float lr, float beta1, float beta2,
                            float eps, float *last_loss);
/* Y (rows x out) = network(X) (device). */
MGEMM_API int32_t mlp_forward(void *mlp, int64_t rows, const float *X, float *Y);
/* idx[r] = argmax over c with M[r,c] != 0 of network(X)[r,c] (lowest index on
 * ties, -1 when no entry is allowed); X, M, idx device. */
MGEMM_API int32_t mlp_predict(void *mlp, int64_t rows, const float *X, const float *M,
                              int32_t *idx);
/* Waits for the library stream and frees the model (NULL is a no-op); returns
 * MGEMM_ERR_HIP if that wait reported an error (the model is freed anyway). */
MGEMM_API int32_t mlp_destroy(void *mlp);

/* Saves a trained network as a tile-configuration model file that
 * mgemm_model_load reads: its parameters (copied from the device), the feature
 * scaling it was trained with and the configuration each output stands for.
 *   path       file to write (replaced);
 *   out_dtype  (host, out entries) dtype of each output, MGEMM_F64 or MGEMM_F32;
 *   out_cfg    (host, out entries) the registered configuration of each output;
 *   feat_mean, feat_std  (host, 6 doubles each, std > 0) the features x = [log2 m,
 *              log2 n, log2 k, dtype == MGEMM_F64, dtype == MGEMM_F32, w] enter the
 *              network as (x - mean) / std rounded to float; w = 1 where the rows of
 *              A and B are whole 16-byte loads (n, lda, ldb multiples of 2 in FP64,
 *              of 4 in FP32; A and B 16-byte aligned), else 0.
 * The network must have 6 inputs.  Every value is written as a C99 hexadecimal
 * float (exact), followed by an FNV-1a checksum of the text.  Returns 0; -1..-6
 * for a NULL argument; MGEMM_ERR_MODEL (not 6 inputs, an output naming a
 * configuration this library does not register, or a failed write). */
MGEMM_API int32_t mlp_save(void *mlp, const char *path, const int32_t *out_dtype,
                           const mgemm_cfg *out_cfg, const double *feat_mean,
                           const double *feat_std);

/* Loads the learned tile-configuration model (a file from mlp_save) for this
 * process, replacing any model loaded before; path NULL unloads.  The paper
 * searches its tuning parameters exhaustively per architecture (Sec. 3, Tab. 4)
 * and names that tuning as the cost that grows with the parameters (Sec. 6); with
 * a model loaded, gemm_ex with cfg == NULL (MGEMM_F64, MGEMM_F32) runs the
 * model's prediction for shapes with m, n, k in [64, 16384] (the range it
 * learned) instead of the built-in table, except where the built-in choice cuts
 * k (split-k: no model output stands for it).  The
 * first such call for a shape evaluates the network on the current device with
 * the library's kernels and waits for it (calls on a stream being captured into a
 * graph use a prediction only if one is already cached);
 * later calls reuse the cached prediction.  The file is read and checked on the
 * host: returns 0, or MGEMM_ERR_MODEL when it cannot be read, its checksum or
 * syntax is wrong, it does not have 6 inputs, or an output names a configuration
 * this library does not register (the model loaded before stays loaded then). */
MGEMM_API int32_t mgemm_model_load(const char *path);

/* The loaded model's configuration for an m x n x k product of dtype stored
 * without padding (lda = k, ldb = n, aligned bases; the output of that dtype
 * with the largest predicted value, lowest index on ties), evaluated by the
 * library's HIP kernels on the current device (the call waits for them;
 * predictions are cached per shape and row class).  Returns 0; -1..-3 (m, n or k
 * below 1), -4 (the model has no output for dtype), -5 (out NULL);
 * MGEMM_ERR_MODEL (no model loaded). */
MGEMM_API int32_t mgemm_model_predict(int64_t m, int64_t n, int64_t k, int32_t dtype,
                                      mgemm_cfg *out);

/* Sets the stream used when a call passes NULL; returns 0. */
MGEMM_API int32_t mgemm_set_stream(void *stream);

/* Text of the last error on this host thread ("" if none).  The pointer stays
 * valid until the next call on this thread. */
MGEMM_API const char *mgemm_last_error(void);

/* Number of registered tile configurations for dtype (negative: bad dtype). */
MGEMM_API int32_t mgemm_config_count(int32_t dtype);

/* Copies registered configuration i of dtype into *out; 0 or -2 / -3. */
MGEMM_API int32_t mgemm_config_get(int32_t dtype, int32_t i, mgemm_cfg *out);

/* What registered configuration i of dtype runs in, as bits: MGEMM_CFG_GEMM
 * (gemm_ex with this cfg), MGEMM_CFG_BATCHED (batched plans accept it),
 * MGEMM_CFG_SPLITK (the built-in choice may cut k with it).  Every registered
 * configuration runs in gemm_ex; the tuning-grid configurations (the paper's
 * tile-size search of Sec. 3, Tab. 4, widened to the GPU's parameters) only there.
 * Returns the bits, -1 (bad dtype) or -2 (i out of range). */
#define MGEMM_CFG_GEMM 1
#define MGEMM_CFG_BATCHED 2
#define MGEMM_CFG_SPLITK 4
MGEMM_API int32_t mgemm_config_flags(int32_t dtype, int32_t i);

/* The tile configuration gemm_ex with cfg == NULL runs for an m x n x k product
 * of dtype (MGEMM_F64 or MGEMM_F32) whose A and B are 16-byte aligned with leading
 * dimensions lda and ldb, on the current device (its compute units enter the
 * choice); a loaded model enters only through the choices it has cached.  *splits
 * receives the number of k ranges (1: k is not cut; above 1 the ranges run the
 * configuration written to *out), *main_rows (main_rows may be NULL) the rows
 * [0, main_rows) that run whole: m without a split, 0 when every row's k is cut,
 * and in between for a split tail (the rows that fill whole rounds of the compute
 * units run whole, the remaining rows with k cut).  For callers that want to know, or to record,
 * what the built-in choice does (the paper fixes its tile parameters per device,
 * Sec. 3, Tab. 4; here they are chosen per product).  Returns 0; -1..-3 (m, n or
 * k below 1), -4 (lda < k), -5 (ldb < n), -6 (dtype), -7 / -8 (out / splits NULL);
 * MGEMM_ERR_NOCONFIG if no configuration is registered. */
MGEMM_API int32_t mgemm_choice(int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                               int32_t dtype, mgemm_cfg *out, int32_t *splits,
                               int64_t *main_rows);

/* Frees the library-owned workspace of the current device (split dtypes and
 * split-k) once the work that last used it has finished; 0 on success,
 * MGEMM_ERR_HIP (workspace kept) if waiting for that work fails. */
MGEMM_API int32_t mgemm_release_workspace(void);

/* Host memory that kernels read and write in place (zero copy), for operands
 * that live in host memory: the counterpart of the paper's comparison of unified
 * (managed) memory with explicit device memory (Sec. 3, the K80 and P100 runs).
 * Page-migrating managed memory needs on-demand GPU page faults, which these
 * GPUs run without; pinned, mapped host memory is the form every kernel can use.
 *   bytes     size of the allocation (> 0);
 *   coherent  1: accesses go to host memory uncached (host writes are seen by a
 *             running kernel); 0: the GPU may cache the memory, and host and
 *             device see each other's writes only at kernel boundaries and
 *             stream synchronisation;
 *   host      receives the host address (for host code);
 *   dev       receives the device address of the same memory (for A, B, C of
 *             any call of this library).
 * The caller owns the memory and frees it with mgemm_host_free(host) once no
 * queued work uses it.  Returns 0; -1 (bytes <= 0) or -2 (NULL out pointer);
 * MGEMM_ERR_HIP if the allocation or its mapping fails (nothing is kept). */
MGEMM_API int32_t mgemm_host_alloc(int64_t bytes, int32_t coherent, void **host, void **dev);

/* Frees memory from mgemm_host_alloc (NULL: no-op); 0 or MGEMM_ERR_HIP. */
MGEMM_API int32_t mgemm_host_free(void *host);

/* Diagnostic: one matrix-core step on one wave with the fragment layout the
 * tiled kernels assume (lane l supplies A[l%16][l/16] and B[l/16][l%16] and
 * receives column l%16 of D; with q = l/16, accumulator element r holds row
 * q+4r for FP64 and row 4q+r for FP32).  dtype is MGEMM_F64 or
 * MGEMM_F32; A (16x4), B (4x16) and D (16x16) are row-major device buffers; on
 * a correct layout D = A*B.  Returns 0, -1 (dtype) or -2 (NULL buffer). */
MGEMM_API int32_t mgemm_probe_mfma(int32_t dtype, const void *A, const void *B, void *D,
                                   void *stream);

/* Diagnostic: one low-precision matrix-core step with operand and accumulator
 * registers passed unchanged per lane, to pin the lane layouts the split path
 * relies on.  kind 0: bf16 32x32x16 (float out), 1: int8 32x32x32 (int32 out),
 * 2: bf16 16x16x32, 3: int8 16x16x64, 4: FP8 e4m3 32x32x64 (float out).  a, b:
 * 64 x 16 bytes of device memory (the 16-byte operand of lane l at byte 16 l; for
 * kind 4 64 x 32 bytes, the 32-byte operand of lane l at byte 32 l); d: 64 x 16
 * 32-bit words (accumulator element r of lane l at word 16 l + r; 4 elements for
 * kinds 2, 3).  Returns 0, -1 (kind) or -2 (NULL buffer). */
MGEMM_API int32_t mgemm_probe_mfma_raw(int32_t kind, const void *a, const void *b, void *d,
                                       void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MGEMM_H */
