// Dense batched training pieces shared by the surrogate network and the NCF model: the BF16
// MFMA GEMM with its epilogues, the weight gradient split over the batch, Adam with its step
// state on the device, the seeded on-device shuffle and the per-step batch rows.  The kernels
// live in mlp.hip; these are their launchers.
#pragma once
#include "common.h"

namespace openk {

// GEMM epilogues: C = A B^T, then
enum {
  EPI_STORE = 0,      // C
  EPI_BIAS = 1,       // C + bias[n]
  EPI_BIAS_GELU = 2,  // Z = C + bias[n] stored, GELU(Z)
  EPI_GELU_GRAD = 3,  // C * GELU'(Z)
  EPI_BIAS_SELU = 4,  // Z = C + bias[n] stored, SELU(Z)
  EPI_SELU_GRAD = 5   // C * SELU'(Z)
};

// Optimizer state on the device, so that a recorded training step can be replayed as is:
// t = Adam steps taken, cursor = batch index within the epoch, c1/c2 = bias corrections of
// the next step, 1 - beta1^(t+1) and 1 - beta2^(t+1).
struct TrainState {
  int64_t t, cursor;
  float c1, c2;
};

// C[m][n] = epilogue(sum_k A(m, k) B(n, k)) with A(m, k) = A[m*sam + k*sak] and
// B(n, k) = Bm[n*sbn + k*sbk], operands rounded to bfloat16, float32 accumulation.
open_status dense_gemm(open_ctx *ctx, const char *name, int epi, int M, int N, int Kd, const float *A, int64_t sam,
                       int64_t sak, const float *Bm, int64_t sbn, int64_t sbk, float *C, int64_t ldc,
                       const float *bias = nullptr, float *Z = nullptr, int64_t ldz = 0);
// g_w[0 .. M*N) = dY^T X and g_w[M*N .. M*N + M) = column sums of dY, over a batch of B rows
// (dY: B x M, X: B x N, row-major), split over the batch into `part` (at least
// dense_wgrad_part_floats(B, M, N) floats) and summed in slice order.
int64_t dense_wgrad_part_floats(int64_t B, int M, int N);
open_status dense_wgrad(open_ctx *ctx, const char *name, int M, int N, int64_t B, const float *dY, const float *X,
                        float *part, float *g_w);
open_status dense_train_state_reset(open_ctx *ctx, TrainState *st);
// Adam (0.9, 0.999, 1e-8, bias-corrected) on np parameters, then the step counter.
open_status dense_adam_step(open_ctx *ctx, int64_t np, float *w, const float *g, float *am, float *av, float lr,
                            TrainState *st);
// loss = sum(part[0..nparts)) / total (float64), to loss_d / loss_f / loss_steps[t] (each nullable)
open_status dense_loss_final(open_ctx *ctx, const double *part, int nparts, int64_t total, double *loss_d,
                             float *loss_f, const TrainState *st, float *loss_steps);
// perm = the seeded order of [0, m) for `epoch` (a Feistel bijection walked along its cycles);
// rewinds the batch cursor
open_status dense_shuffle(open_ctx *ctx, int64_t m, uint64_t seed, int64_t epoch, int64_t *perm, TrainState *st);
// rows[t] = perm[cursor * batch + t]
open_status dense_rows_of_step(open_ctx *ctx, const int64_t *perm, int batch, const TrainState *st, int64_t *rows);

}  // namespace openk
