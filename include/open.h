/*
 * open.h -- C ABI of the MI355X collaborative-filtering hot path of OPEN
 * (online performance prediction under CPU and GPU power caps).
 *
 * The paper completes a sparse application x power-setting performance matrix from a few
 * profiled entries of each new application (Section III-B.1 and III-B.2; the matrix of
 * Eq. 1 gains one sparse row per new application) and then picks the energy-efficient
 * CPU/GPU cap pair of each application with Algorithm 2 (Section III-B.3).  This library
 * completes the matrix by weighted-lambda alternating least squares (the CF formulation
 * of the paper's Netflix-prize reference, Zhou et al. 2008, cited in Section III-B.1),
 * folds new rows in against fixed setting factors, predicts, and selects.
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major float32; rows are applications, columns are settings.
 *     A setting index is s = a * n_gpu + b for CPU-cap index a and GPU-cap index b.
 *   - Sparse inputs are CSR: row_ptr int64[m+1] (row_ptr[0] = 0), col int32[nnz] sorted and
 *     unique within each row and in [0, n), val float32[nnz].
 *   - Unless stated otherwise every pointer is a DEVICE pointer owned by the caller.  The
 *     library never frees caller memory and never returns memory it allocated; its own
 *     workspaces live in the context and are reused across calls.
 *   - Calls are asynchronous on the context's stream unless they return a host value.
 *   - Invalid arguments return OPEN_E_INVALID before any work is queued; the message is
 *     available from open_last_error().  No C++ exception crosses this interface.
 *   - Per-row numerical failures do not abort a call: the row's output is zero, its
 *     row_status entry is set and the call returns OPEN_OK; callers inspect row_status.
 *   - Supported ranks k: 8, 16, 32, 64.  Other ranks return OPEN_E_UNSUPPORTED.
 *   - One context serves one host thread at a time.  Results are deterministic: repeated
 *     calls on the same inputs return bitwise identical outputs.
 */
#ifndef OPEN_H
#define OPEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct open_ctx open_ctx;
typedef struct open_mlp open_mlp;

typedef enum {
  OPEN_OK = 0,
  OPEN_E_INVALID = -1,     /* bad shape, pointer, option or rank */
  OPEN_E_NOMEM = -2,       /* a workspace allocation failed */
  OPEN_E_DEVICE = -3,      /* a HIP runtime call failed */
  OPEN_E_UNSUPPORTED = -4  /* valid request this build does not implement (e.g. rank 12) */
} open_status;

/* row_status values */
enum {
  OPEN_ROW_OK = 0,
  OPEN_ROW_EMPTY = 1,         /* no observed entry: output row is zero */
  OPEN_ROW_NONPOS_PIVOT = 2,  /* system not positive definite in float32 (e.g. lambda = 0) */
  OPEN_ROW_NONFINITE = 3,     /* an observed value is NaN or infinite */
  OPEN_ROW_NONPOS_BASE = 4,   /* Alg. 2: predicted baseline performance not positive */
  OPEN_ROW_BADINDEX = 5       /* a column index outside [0, n): output row is zero */
};

/* Context on `device` (HIP ordinal), issuing work on `hip_stream` (a hipStream_t; NULL = the
 * null stream).  On success *ctx owns the device workspaces until open_destroy. */
open_status open_create(open_ctx **ctx, int device, void *hip_stream);
open_status open_destroy(open_ctx *ctx);
/* Rebind the context to another stream of the same device. */
open_status open_set_stream(open_ctx *ctx, void *hip_stream);
/* Last error message of the context (static storage owned by the context; never NULL). */
const char *open_last_error(const open_ctx *ctx);
/* Block until the context's stream has drained. */
open_status open_sync(open_ctx *ctx);

/* Per-kernel timing: when enabled, every kernel the context launches is bracketed by HIP
 * events on its stream.  open_profile_read drains the stream and reports, per kernel name
 * (static strings owned by the library), the summed duration in milliseconds and the launch
 * count; it returns the number of distinct kernels (entries beyond `max` are dropped) or -1
 * on error, and forgets the records when reset != 0. */
open_status open_profile(open_ctx *ctx, int32_t enable);
int32_t open_profile_read(open_ctx *ctx, const char **names, double *total_ms, int64_t *launches, int32_t max,
                          int32_t reset);

/*
 * Fold-in (Section III-B.2: a new application's few profiled entries become a sparse row
 * whose missing entries collaborative filtering fills).  With the setting factors F (n x k)
 * fixed, every CSR row i (m rows) gets the ridge solution
 *     u_i = (sum_{j in O_i} f_j f_j^T + lambda w_i I)^-1  sum_{j in O_i} r_ij f_j,
 * w_i = |O_i| when weighted != 0 (ALS-WR weighting) and 1 otherwise.  The same call is the
 * row half-sweep of ALS (F = V, rows = applications) and the column half-sweep (F = U, the
 * CSR being the column view of the matrix).  Rows with |O_i| <= min(k, 32) are solved in the
 * dual form u = F_O^T (F_O F_O^T + lambda w I)^-1 r, the same number.
 *   F          device float32[n*k]
 *   U_out      device float32[m*k], written
 *   row_status device int32[m] or NULL
 * lambda must be >= 0 and finite. */
open_status open_foldin(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m, const int64_t *row_ptr,
                        const int32_t *col, const float *val, float lambda, int32_t weighted, float *U_out,
                        int32_t *row_status);

/*
 * Fold-in through a HIP graph: the same result as open_foldin (same kernels, same order).
 * The first call with a given set of arguments runs eagerly and records the launch sequence
 * into a graph held by the context; a later call with identical pointers, sizes, lambda,
 * weighting and kernel-variant choice replays it with one hipGraphLaunch (the values behind
 * the pointers may change between calls).  Other arguments re-record.  Only the sync-free
 * fold-in can be recorded: rank 8, 16 or 32 and n < 1024 (else OPEN_E_UNSUPPORTED).
 */
open_status open_foldin_graph(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m,
                              const int64_t *row_ptr, const int32_t *col, const float *val, float lambda,
                              int32_t weighted, float *U_out, int32_t *row_status);

/*
 * Allocation-free fold-in, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, same
 * kernels and the same result as open_foldin, bit for bit, but the bucketing buffers live in
 * a static device array of the library (about 16 MiB per GPU, held until the process ends)
 * instead of context workspaces, so the call allocates nothing, frees nothing and never waits
 * on the host.
 *   Limits: m <= open_foldin_noalloc_max_rows() (1,048,576) rows per call, else
 *   OPEN_E_INVALID; n < 1024 factor rows (no split-K rows), else OPEN_E_UNSUPPORTED.
 *   Sharing: every call on one GPU uses that GPU's one array, which keeps the last call's
 *   contents (each call writes every element it reads).  Calls that overlap in time on one
 *   GPU (other streams, other contexts, other host threads) race; serialize them.
 */
open_status open_foldin_noalloc(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m,
                                const int64_t *row_ptr, const int32_t *col, const float *val, float lambda,
                                int32_t weighted, float *U_out, int32_t *row_status);
int64_t open_foldin_noalloc_max_rows(void);

/*
 * Phase-transition detection (Algorithm 1, Section III-B.2) for T power traces at once.
 * Trace t is power[t*ld .. t*ld + L) (device float32, GPU power readings in W at a fixed
 * sampling interval).  first_index[t] (device int64) receives the 0-based index of the
 * reading at which the last n_window readings are all >= threshold (the paper: 0.2 s
 * sampling, 5 s window -> n_window = 25, threshold 60 W), or -1 if that never happens.
 * The comparison is literal ("below threshold" breaks the condition), so NaN readings do
 * not.  Integer result, independent of scheduling.  OPEN_E_INVALID for T < 0, L < 0,
 * ld < L, n_window < 1 or a NaN threshold.
 */
open_status open_phase_detect(open_ctx *ctx, const float *power, int64_t T, int64_t L, int64_t ld, float threshold,
                              int32_t n_window, int64_t *first_index);

/*
 * Kernel variants and autotuning (the fold-in's batched solves, Section III-B.2, run one
 * kernel per size class of |O_i|; each class group has up to 4 compiled configurations:
 * lanes per system, waves per block, waves per SIMD).  The choice is per context and rank
 * and applies to every later call that solves ridge rows (open_foldin, open_fit, the
 * surrogate fallback).
 *
 * open_tune_info: number of class groups of rank k (8, 16, 32, 64; -1 otherwise); for the
 *   first `max` groups, names[g] (static strings) and nvar[g] (variants compiled), either
 *   array may be NULL.
 * open_tune_get / open_tune_set: the chosen variant per group, host int8[count]; set
 *   rejects a value outside [0, nvar) with OPEN_E_INVALID and changes nothing then.
 * open_autotune: the arguments of open_foldin plus `reps` (>= 1 timed launches per
 *   variant after one untimed one).  Buckets the batch once, times every variant of each
 *   group that holds rows, keeps the fastest, and leaves the fold-in result of the chosen
 *   variants in U_out (and row_status).  Groups without rows keep their choice.  ms_out
 *   (host float64[groups * 4] or NULL) receives milliseconds per launch, -1 where untimed.
 *   Synchronises the stream.
 */
int32_t open_tune_info(int32_t k, const char **names, int32_t *nvar, int32_t max);
open_status open_tune_get(open_ctx *ctx, int32_t k, int8_t *choice, int32_t count);
open_status open_tune_set(open_ctx *ctx, int32_t k, const int8_t *choice, int32_t count);
open_status open_autotune(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m, const int64_t *row_ptr,
                          const int32_t *col, const float *val, float lambda, int32_t weighted, float *U_out,
                          int32_t *row_status, int32_t reps, double *ms_out);

/*
 * Warm-started refit (Section III-B.2: new applications expand the matrix, which is then
 * completed): the CSR holds the m_old offline rows first, then the m_new new rows.  U
 * (device, (m_old + m_new) x k) holds the fitted offline factors in its first m_old rows on
 * entry; V (n x k) the fitted setting factors.  The new rows are folded in against V
 * (open_foldin), then `sweeps` ALS-WR sweeps run on the union (open_fit, same conventions),
 * updating U and V.  sweeps = 0 leaves the plain fold-in.
 */
open_status open_refit(open_ctx *ctx, int64_t m_old, int64_t m_new, int32_t n, int32_t k, const int64_t *row_ptr,
                       const int32_t *col, const float *val, float lambda, int32_t weighted, int32_t sweeps, float *U,
                       float *V, double *obj_hist);

/*
 * Column view of a CSR matrix (m x n): col_ptr int64[n+1], row_idx int32[nnz] and
 * cval float32[nnz], entries ordered by column and, within a column, by row.  Exact
 * integer work (a stable counting sort).  All pointers are device pointers.
 */
open_status open_csr_to_csc(open_ctx *ctx, int64_t m, int32_t n, const int64_t *row_ptr, const int32_t *col,
                            const float *val, int64_t *col_ptr, int32_t *row_idx, float *cval);

/*
 * ALS-WR fit (weighted-lambda alternating least squares): `sweeps` times, every row against
 * V (open_foldin on the CSR), then every column against U (open_foldin on the column view).
 * A column with no observation gets v_j = 0.  U (m*k) and V (n*k) hold the initial factors
 * on entry and the fitted factors on return.  obj_hist, when not NULL, is a HOST array of
 * 2*sweeps doubles receiving the objective
 *     f = sum_O (r_ij - u_i.v_j)^2 + lambda (sum_i w_i |u_i|^2 + sum_j w^j |v_j|^2)
 * after every half-sweep; it makes the call synchronous.  Rows and columns with at least 1024
 * observed entries are solved by the split-K path (chunked Gram matrices, reduced in chunk
 * order); rank 64 supports up to 32 and from 1024 observed entries per row or column.
 * Without obj_hist and with sweeps >= 2, the first sweep runs eagerly and the others replay
 * it as one HIP graph (the same kernels in the same order).  The call returns after its
 * temporary buffers are released, so it drains the stream.
 */
open_status open_fit(open_ctx *ctx, int64_t m, int32_t n, int32_t k, const int64_t *row_ptr, const int32_t *col,
                     const float *val, float lambda, int32_t weighted, int32_t sweeps, float *U, float *V,
                     double *obj_hist);

/* Objective f(U, V) above, reduced in float64 in a fixed order; *out is a HOST double.
 * Synchronous. */
open_status open_objective(open_ctx *ctx, int64_t m, int32_t n, int32_t k, const int64_t *row_ptr,
                           const int32_t *col, const float *val, const float *U, const float *V, float lambda,
                           int32_t weighted, double *out);

/* Observed-entry RMS residual of every row, rho_i = sqrt(mean_{j in O_i} (r_ij - u_i.v_j)^2)
 * (0 for an empty row).  rho: device float32[m]. */
open_status open_residual(open_ctx *ctx, int64_t m, int32_t n, int32_t k, const int64_t *row_ptr,
                          const int32_t *col, const float *val, const float *U, const float *V, float *rho);

/*
 * Fused predict + Algorithm 2 (Section III-B.3).  p_is = u_i . v_s for all s; with the
 * baseline setting `base` = (C_b, G_b), E_base = C_b + G_b; setting s is valid when p_is > 0
 * and 1 - p_is / p_ib <= gamma; its energy bound is E_s = (c_s + g_s) / p_is; the valid
 * setting of least E_s (greatest saving (E_base - E_s) / E_base) wins, the lowest s on ties.
 * In float32 the validity test is evaluated exactly as written (correctly rounded division);
 * the least E_s is taken as the greatest p_is * fl(1 / (c_s + g_s)), and the saving from
 * E_s = fl((c_s + g_s) / p_is) of the winner.
 *   U          device float32[m*k];  V device float32[n*k]
 *   cap_cpu, cap_gpu  device float32[n], watts of setting s (c_s + g_s finite and positive)
 *   P          device float32[m*n] or NULL (the full prediction is only written when asked)
 *   best_idx   device int32[m]; best_saving device float32[m] or NULL
 *   row_status device int32[m] or NULL (OPEN_ROW_NONPOS_BASE when p_ib <= 0; then
 *              best_idx = base and saving = 0)
 */
open_status open_predict(open_ctx *ctx, const float *U, int64_t m, const float *V, int32_t n, int32_t k, float *P,
                         const float *cap_cpu, const float *cap_gpu, int32_t base, float gamma, int32_t *best_idx,
                         float *best_saving, int32_t *row_status);

/*
 * Fold-in surrogate: a network that maps a new application's masked profile vector
 * x = [r * mask ; mask] (length 2n) straight to its latent row,
 *     h1 = GELU(W1 x + b1),  h2 = GELU(W2 h1 + b2),  u = W3 h2 + b3,
 * GELU(z) = z/2 (1 + erf(z/sqrt 2)), trained on ridge fold-ins and backed by them: a row
 * whose observed-entry RMS residual exceeds tau is re-solved by open_foldin.  Weights are
 * kept in float32 (the master copy Adam updates) and used as bfloat16 (round to nearest
 * even) in the matrix products, which accumulate in float32.
 *
 * Parameter packing (host float32 arrays, this order, row-major):
 *   W1[hidden][2n], b1[hidden], W2[hidden][hidden], b2[hidden], W3[k][hidden], b3[k].
 * hidden must be 256; n at most 4096.
 */
/* init_host: HOST float32 weights in that packing, or NULL for seeded weights: every weight
 * and bias of a layer with fan-in f uniform on [-1/sqrt f, 1/sqrt f), parameter e of the
 * flat vector drawn as (mix64(seed ^ mix64(e)) >> 40) * 2^-24 in [0, 1), mix64 being the
 * SplitMix64 output function (Steele, Lea and Flood 2014). */
open_status open_mlp_create(open_ctx *ctx, open_mlp **mlp, int32_t n, int32_t k, int32_t hidden,
                            const float *init_host, uint64_t seed);
open_status open_mlp_destroy(open_mlp *mlp);
/* Number of float32 parameters in the packing above. */
int64_t open_mlp_num_params(int32_t n, int32_t k, int32_t hidden);
/* Copy the float32 master weights to a HOST array (packing above).  Synchronous. */
open_status open_mlp_get_weights(open_mlp *mlp, float *host_out);
/* Replace the master weights from a HOST array; resets the Adam state and step count. */
open_status open_mlp_set_weights(open_mlp *mlp, const float *host_in);

/* Network output for every CSR row: U_hat device float32[m*k]. */
open_status open_mlp_forward(open_mlp *mlp, int64_t m, const int64_t *row_ptr, const int32_t *col,
                             const float *val, float *U_hat);

/* Loss L = 1/(B k) sum |u_hat_i - target_i|^2 over the B = m rows of the CSR and its gradient
 * with respect to every parameter (packing above), written to the HOST arrays *loss and
 * grads_host.  Does not update the weights.  Synchronous.  m <= 16384. */
open_status open_mlp_loss_grad(open_mlp *mlp, int64_t m, const int64_t *row_ptr, const int32_t *col,
                               const float *val, const float *target, double *loss, float *grads_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the batch formed by
 * the CSR rows listed in rows[0..batch) (device int64; NULL = rows 0..batch-1) with targets
 * target[rows[b]*k ..].  loss_out: device float32 scalar or NULL.  m is the CSR row count. */
open_status open_mlp_train_step(open_mlp *mlp, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                const float *val, const float *target, const int64_t *rows, int32_t batch,
                                float lr, float *loss_out);

/* Training: `epochs` passes over the m CSR rows with their targets (device float32[m*k]), each
 * epoch in a new seeded order, m / batch full batches per epoch (the remainder waits for a
 * later order), one Adam step per batch exactly as open_mlp_train_step takes it.  The order of
 * epoch e is a permutation computed on the device: a four-round Feistel network on 2h-bit
 * integers (4^h >= m), round keys mix64(mix64(seed) + 4e + r), round function mix64(R ^ key)
 * masked to h bits, walked along its cycle until the value is below m.  The first step runs
 * eagerly and the step sequence is then replayed as one recorded HIP graph.  loss_hist: HOST
 * float32[epochs] or NULL, the mean batch loss of each epoch.  Synchronous.
 * batch in [1, min(16384, m)]; epochs >= 0; lr finite and > 0. */
open_status open_mlp_train(open_mlp *mlp, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *val,
                           const float *target, int32_t batch, float lr, int32_t epochs, uint64_t seed,
                           float *loss_hist);

/* Surrogate fold-in with ridge fallback: u_i = network output unless its observed-entry RMS
 * residual against the setting factors F exceeds tau, in which case u_i is the ridge
 * solution of open_foldin (lambda, weighted).  used_fallback (device uint8[m] or NULL)
 * marks re-solved rows; rho (device float32[m] or NULL) receives the network's residual;
 * n_fallback (HOST int64, or NULL) receives the number of re-solved rows and makes the
 * call synchronous. */
open_status open_mlp_foldin(open_mlp *mlp, const float *F, int64_t m, const int64_t *row_ptr, const int32_t *col,
                            const float *val, float tau, float lambda, int32_t weighted, float *U_out,
                            uint8_t *used_fallback, float *rho, int64_t *n_fallback);

/*
 * Offline performance predictor (Section III-A.2, "Performance Prediction Model"), batched
 * over n_runs profiled runs.  Run r's seven features X[r*7 .. r*7+7) (device float32, in the
 * order CPU power cap, GPU power cap, memory throughput, IPS, SM clock, DRAM active rate,
 * FP active rate) give its predicted normalized performance y[r] (device float32[n_runs]):
 *   z = (x - mu) * rs,  h1 = ReLU(W1 z + b1),  h2 = ReLU(W2 h1 + b2),  y = w3 . h2 + b3,
 * mu, rs: device float32[7] (feature centring and inverse scale); W1 float32[64*7] and
 * W2 float32[64*64] row-major (output unit major), used rounded to bfloat16 (nearest even);
 * b1, b2, w3 float32[64]; b3 float32[1]; all on the device and owned by the caller.  The
 * activations keep float32 precision (products of the bfloat16 weights with two-part
 * activations, float32 accumulation).  A run with a non-finite feature gets y = NaN.
 * Asynchronous on the context's stream.  OPEN_E_INVALID
 * for n_runs < 0 or a null pointer (n_runs = 0 does nothing).
 */
open_status open_perf_predict(open_ctx *ctx, const float *X, int64_t n_runs, const float *mu, const float *rs,
                              const float *W1, const float *b1, const float *W2, const float *b2, const float *w3,
                              const float *b3, float *y);

/*
 * Neural collaborative filtering fold-in (Section III-B.1 model; Section III-B.2, the new
 * application's missing entries are imputed by the CF model).  The model scores application
 * embedding e against setting embedding s_j:
 *   y(e, s_j) = w3 . SELU(W2 SELU(W1 [e; s_j] + b1) + b2) + b3,
 * SELU(z) = lambda (z if z > 0 else alpha (exp(z) - 1)), alpha = 1.6732632..., lambda =
 * 1.0507009....  For each CSR row i (observed settings col, values val) the embedding E_out[i]
 * is learned with S and the network fixed: `steps` steps of gradient descent from e = 0 with
 * step eta on L(e) = (1/q) sum_j (y(e, s_j) - r_ij)^2 + mu |e|^2 (q = entries of the row).
 *   S        device float32[n*d] setting embeddings, d = 32 (else OPEN_E_UNSUPPORTED)
 *   W1       device float32[64*2d] row-major (unit major; the first d inputs are e); b1[64]
 *   W2       device float32[64*64]; b2[64]; w3[64]; b3[1]
 *   E_out    device float32[m*d], written; loss_out device float32[m] or NULL: L(e) at the
 *            returned e; row_status device int32[m] or NULL.
 * Rows with no entry (status 1), a column outside [0, n) (status 5) or a non-finite value
 * (status 3) keep e = 0 and loss 0.  Float32 arithmetic.  OPEN_E_INVALID for n < 1, m < 0,
 * steps outside [0, 100000], NaN eta or mu, or a null pointer.  Asynchronous on the context's
 * stream.
 */
open_status open_ncf_foldin(open_ctx *ctx, const float *S, int32_t n, int32_t d, const float *W1, const float *b1,
                            const float *W2, const float *b2, const float *w3, const float *b3, int64_t m,
                            const int64_t *row_ptr, const int32_t *col, const float *val, int32_t steps, float eta,
                            float mu, float *E_out, float *loss_out, int32_t *row_status);

/*
 * NCF offline training (Section III-B.1: the CF model learns from the profiled applications):
 * the model above, application embeddings E included, fitted to a dense offline matrix R
 * (m_off applications x n settings, every entry observed) by Adam (0.9, 0.999, 1e-8,
 * bias-corrected) on the mean squared error over batches of whole applications (each batch
 * entry pairs an application with one of its settings).  Epoch e visits the applications in
 * the seeded device order that open_mlp_train uses (Feistel network, keys from seed and e);
 * m_off / apps_per_batch batches per epoch.  The products run on BF16 MFMA with float32
 * accumulation (float32 masters); the embedding gradients are summed in a fixed order.
 *   R        device float32[m_off*n] row-major
 *   params   device float32[open_ncf_num_params(m_off, n)], in/out, packed as
 *            E[m_off][d], S[n][d], W1[64][2d], b1[64], W2[64][64], b2[64], w3[64], b3[1]
 *            (d = 32); S, W1 ... b3 are the arguments of open_ncf_foldin
 *   loss_hist HOST float32[epochs] or NULL: mean batch loss of each epoch
 * apps_per_batch in [1, m_off] with apps_per_batch * n <= 2^20.  Synchronous.
 */
int64_t open_ncf_num_params(int64_t m_off, int32_t n);
open_status open_ncf_train(open_ctx *ctx, int64_t m_off, int32_t n, int32_t d, const float *R, float *params,
                           int32_t apps_per_batch, float lr, int32_t epochs, uint64_t seed, float *loss_hist);
/* Loss and gradient (HOST float32[open_ncf_num_params], same packing) of one batch: the G
 * distinct applications listed in apps (device int64[G]) with all n settings each; the
 * parameters are not changed.  Synchronous. */
open_status open_ncf_loss_grad(open_ctx *ctx, int64_t m_off, int32_t n, int32_t d, const float *R,
                               const float *params, const int64_t *apps, int32_t G, double *loss, float *grads_host);

#ifdef __cplusplus
}
#endif
#endif /* OPEN_H */
