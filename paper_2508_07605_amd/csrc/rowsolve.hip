// Dispatch of the batched ridge solves to the size-class kernels of each rank, the kernel
// variant table, and the autotuner that picks a variant per class group by timing.
#include <string.h>

#include <vector>

#include "rowsolve.h"

namespace openk {

const ClassGroup *class_groups(int k, int *count) {
  static const ClassGroup g8[] = {
      {"ridge_k8_d4", 0, 1, 2, g_k8_d4},
      {"ridge_k8_d8", 2, 2, 2, g_k8_d8},
      {"ridge_k8_primal", 9, 15, 2, g_k8_primal},
  };
  static const ClassGroup g16[] = {
      {"ridge_k16_d4", 0, 1, 2, g_k16_d4},
      {"ridge_k16_d8", 2, 2, 2, g_k16_d8},
      {"ridge_k16_d12", 3, 3, 2, g_k16_d12},
      {"ridge_k16_d16", 4, 4, 2, g_k16_d16},
      {"ridge_k16_primal", 9, 15, 2, g_k16_primal},
  };
  static const ClassGroup g32[] = {
      {"ridge_k32_d4", 0, 1, 2, g_k32_d4},
      {"ridge_k32_d8", 2, 2, 2, g_k32_d8},
      {"ridge_k32_d12", 3, 3, 2, g_k32_d12},
      {"ridge_k32_d16", 4, 4, 4, g_k32_d16},
      {"ridge_k32_d20", 5, 5, 4, g_k32_d20},
      {"ridge_k32_d24", 6, 6, 4, g_k32_d24},
      {"ridge_k32_d28", 7, 7, 2, g_k32_d28},
      {"ridge_k32_d32", 8, 8, 2, g_k32_d32},
      {"ridge_k32_primal", 9, 15, 2, g_k32_primal},
      // launch mode of the whole pass: 0 = three merged launches, 1 = one launch per group above
      {"ridge_k32_launch", 0, 15, 2, nullptr},
  };
  static const ClassGroup g64[] = {
      {"ridge_k64_d4", 0, 1, 2, g_k64_d4},
      {"ridge_k64_d8", 2, 2, 2, g_k64_d8},
      {"ridge_k64_d12", 3, 3, 2, g_k64_d12},
      {"ridge_k64_d16", 4, 4, 2, g_k64_d16},
      {"ridge_k64_d20", 5, 5, 2, g_k64_d20},
      {"ridge_k64_d24", 6, 6, 2, g_k64_d24},
      {"ridge_k64_d28", 7, 7, 2, g_k64_d28},
      {"ridge_k64_d32", 8, 8, 2, g_k64_d32},
      {"ridge_k64_primal", 9, 15, 1, g_k64_primal},
  };
  switch (k) {
    case 8: *count = (int)(sizeof(g8) / sizeof(g8[0])); return g8;
    case 16: *count = (int)(sizeof(g16) / sizeof(g16[0])); return g16;
    case 32: *count = (int)(sizeof(g32) / sizeof(g32[0])); return g32;
    case 64: *count = (int)(sizeof(g64) / sizeof(g64[0])); return g64;
    default: *count = 0; return nullptr;
  }
}

int rank_index(int k) { return k == 8 ? 0 : k == 16 ? 1 : k == 32 ? 2 : k == 64 ? 3 : -1; }

// The launch mode of the rank: its last table entry when that is a group without a kernel,
// else 1 (one launch per class group).
static int launch_mode(const open_ctx *ctx, int k, const ClassGroup *g, int ng) {
  return (k == 32 && ng > 0 && !g[ng - 1].fn) ? ctx->tune[rank_index(k)][ng - 1] : 1;
}

open_status rowsolve_launch(open_ctx *ctx, const float *F, int n, int k, const int64_t *ptr, const int32_t *idx,
                            const float *val, float lambda, int weighted, const RowRef *list, const int64_t *cls,
                            float *X, int32_t *status, int64_t m) {
  int ng = 0;
  const ClassGroup *g = class_groups(k, &ng);
  if (!g) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  const int ri = rank_index(k);
  if (launch_mode(ctx, k, g, ng) == 0) return rowsolve_k32_merged(OPEN_TIER_PASS, X, status, m);
  for (int i = 0; i < ng; ++i) {
    if (!g[i].fn) continue;
    open_status st = g[i].fn(ctx->tune[ri][i], OPEN_TIER_PASS, X, status, m);
    if (st) return st;
  }
  return OPEN_OK;
}

// Time every variant of every populated class group on one bucketed batch (reps launches
// each, after one untimed launch) and keep the fastest per group.
open_status rowsolve_autotune(open_ctx *ctx, const float *F, int n, int k, const int64_t *ptr, const int32_t *idx,
                              const float *val, float lambda, int weighted, const RowRef *list, const int64_t *cls,
                              float *X, int32_t *status, int64_t m, int reps, double *ms_out) {
  int ng = 0;
  const ClassGroup *g = class_groups(k, &ng);
  if (!g) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  const int ri = rank_index(k);
  int64_t *h;
  open_status st;
  if ((st = pinned_get(ctx, sizeof(int64_t) * 2 * kNumClasses, (void **)&h))) return st;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, cls, sizeof(int64_t) * 2 * kNumClasses, hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<int64_t> rows(ng, 0);
  for (int i = 0; i < ng; ++i)
    for (int c = g[i].c_lo; c <= g[i].c_hi; ++c) rows[i] += h[2 * c + 1];
  hipEvent_t e0, e1;
  OPEN_HIP_TRY(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, OPEN_E_DEVICE, "hipEventCreate failed");
  }
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  for (int i = 0; i < ng && st == OPEN_OK; ++i) {
    if (ms_out)
      for (int v = 0; v < kMaxVariants; ++v) ms_out[i * kMaxVariants + v] = -1.0;
    if (rows[i] == 0 || !g[i].fn) continue;
    int best = ctx->tune[ri][i];
    double best_ms = 0.0;
    for (int v = 0; v < g[i].nvar && v < kMaxVariants && st == OPEN_OK; ++v) {
      if ((st = g[i].fn(v, OPEN_TIER_PASS, X, status, m))) break;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) st = fail(ctx, OPEN_E_DEVICE, "hipEventRecord failed");
      for (int r = 0; r < reps && st == OPEN_OK; ++r) st = g[i].fn(v, OPEN_TIER_PASS, X, status, m);
      if (st) break;
      float ms = 0.f;
      if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(ctx, OPEN_E_DEVICE, "event timing failed");
        break;
      }
      const double per = (double)ms / reps;
      if (ms_out) ms_out[i * kMaxVariants + v] = per;
      if (v == 0 || per < best_ms) {
        best_ms = per;
        best = v;
      }
    }
    if (st == OPEN_OK) ctx->tune[ri][i] = (int8_t)best;
  }
  // the launch mode: the whole pass in each mode, with the variants just chosen
  if (st == OPEN_OK && ng > 0 && !g[ng - 1].fn) {
    const int li = ng - 1;
    int best = 0;
    double best_ms = 0.0;
    for (int v = 0; v < g[li].nvar && v < kMaxVariants && st == OPEN_OK; ++v) {
      ctx->tune[ri][li] = (int8_t)v;
      if ((st = rowsolve_launch(ctx, F, n, k, ptr, idx, val, lambda, weighted, list, cls, X, status, m))) break;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) st = fail(ctx, OPEN_E_DEVICE, "hipEventRecord failed");
      for (int r = 0; r < reps && st == OPEN_OK; ++r)
        st = rowsolve_launch(ctx, F, n, k, ptr, idx, val, lambda, weighted, list, cls, X, status, m);
      if (st) break;
      float ms = 0.f;
      if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(ctx, OPEN_E_DEVICE, "event timing failed");
        break;
      }
      const double per = (double)ms / reps;
      if (ms_out) ms_out[li * kMaxVariants + v] = per;
      if (v == 0 || per < best_ms) {
        best_ms = per;
        best = v;
      }
    }
    ctx->tune[ri][li] = (int8_t)best;
  }
  ctx->prof_on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  // leave the result of the chosen variants in X
  return rowsolve_launch(ctx, F, n, k, ptr, idx, val, lambda, weighted, list, cls, X, status, m);
}

}  // namespace openk
