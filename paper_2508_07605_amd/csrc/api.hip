// C ABI entry points of libopen: argument validation, context and workspace management,
// dispatch to the kernels.  See include/open.h for the contract of every call.
#include <limits.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <functional>
#include <mutex>
#include <new>
#include <string>

#include "common.h"
#include "rowsolve.h"

namespace openk {

// ---- static scratch of the allocation-free fold-in (one copy per GPU, held until the process
// ends).  Layout: the bucketed row list, then the per-block class counts, then the class table.
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 20;
constexpr size_t kScrList = 0;
constexpr size_t kScrHist = kScrList + sizeof(RowRef) * (size_t)kNoAllocMaxRows;
constexpr size_t kScrCls = kScrHist + ((sizeof(int32_t) * (size_t)kNumClasses * (size_t)(kNoAllocMaxRows / kBucketRowsPerBlock) + 255) &
                                       ~(size_t)255);
constexpr size_t kScrBytes = kScrCls + sizeof(int64_t) * 2 * kNumClasses;
static __device__ __align__(256) unsigned char scratch[kScrBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device with the device
// current.  The array's name in host code is not a device address.
static hipError_t scratch_address(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_addr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

open_status ws_get(open_ctx *ctx, int slot, size_t bytes, void **out) {
  if (bytes == 0) bytes = 16;
  if (ctx->ws_bytes[slot] < bytes && ctx->capturing)
    return fail(ctx, OPEN_E_UNSUPPORTED, "workspace growth during graph capture");
  if (ctx->ws_bytes[slot] < bytes) {
    if (ctx->ws[slot]) {
      // the stream may still use the old buffer: drain before releasing it
      OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      OPEN_HIP_TRY(ctx, hipFree(ctx->ws[slot]));
      ctx->ws[slot] = nullptr;
      ctx->ws_bytes[slot] = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&ctx->ws[slot], want) != hipSuccess) {
      (void)hipGetLastError();
      ctx->ws[slot] = nullptr;
      return fail(ctx, OPEN_E_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->ws_bytes[slot] = want;
    ++ctx->ws_gen;
  }
  *out = ctx->ws[slot];
  return OPEN_OK;
}

open_status pinned_get(open_ctx *ctx, size_t bytes, void **out) {
  if (ctx->capturing) return fail(ctx, OPEN_E_UNSUPPORTED, "host read-back during graph capture");
  if (ctx->host_pinned_bytes < bytes) {
    if (ctx->host_pinned) {
      OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      OPEN_HIP_TRY(ctx, hipHostFree(ctx->host_pinned));
      ctx->host_pinned = nullptr;
      ctx->host_pinned_bytes = 0;
    }
    OPEN_HIP_TRY(ctx, hipHostMalloc(&ctx->host_pinned, bytes, hipHostMallocDefault));
    ctx->host_pinned_bytes = bytes;
  }
  *out = ctx->host_pinned;
  return OPEN_OK;
}

static hipEvent_t prof_event(open_ctx *ctx) {
  if (ctx->prof_pool_used == ctx->prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->prof_pool.push_back(e);
  }
  return ctx->prof_pool[ctx->prof_pool_used++];
}

void prof_begin(open_ctx *ctx, const char *name) {
  if (!ctx->prof_on) return;
  open_ctx::ProfRec r{name, prof_event(ctx), prof_event(ctx)};
  if (r.beg && r.end) {
    (void)hipEventRecord(r.beg, ctx->stream);
    ctx->prof_recs.push_back(r);
  }
}

void prof_end(open_ctx *ctx) {
  if (!ctx->prof_on || ctx->prof_recs.empty()) return;
  (void)hipEventRecord(ctx->prof_recs.back().end, ctx->stream);
}

static bool rank_ok(int k) { return k == 8 || k == 16 || k == 32 || k == 64; }

// Validate a CSR header shared by several calls.
static open_status check_csr(open_ctx *ctx, int64_t m, const int64_t *row_ptr, const int32_t *col,
                             const float *val) {
  if (m < 0 || m >= INT_MAX) return fail(ctx, OPEN_E_INVALID, "row count must be in [0, 2^31 - 1)");
  if (m > 0 && (!row_ptr || !col || !val)) return fail(ctx, OPEN_E_INVALID, "CSR pointers must not be NULL");
  return OPEN_OK;
}

// Capture the launches of fn() on a private stream into a graph (nothing runs).
open_status graph_capture(open_ctx *ctx, const std::function<open_status()> &fn, hipGraph_t *out) {
  *out = nullptr;
  if (!ctx->cap_stream) OPEN_HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t user = ctx->stream;
  const bool prof = ctx->prof_on;
  OPEN_HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  ctx->stream = ctx->cap_stream;
  ctx->capturing = true;
  ctx->prof_on = false;
  open_status st = fn();
  ctx->stream = user;
  ctx->capturing = false;
  ctx->prof_on = prof;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || !g) {
    (void)hipGetLastError();
    return fail(ctx, OPEN_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  *out = g;
  return OPEN_OK;
}

}  // namespace openk

using namespace openk;

extern "C" {

open_status open_create(open_ctx **out, int device, void *hip_stream) {
  if (!out) return OPEN_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return OPEN_E_DEVICE;
  }
  open_ctx *ctx = new (std::nothrow) open_ctx();
  if (!ctx) return OPEN_E_NOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return OPEN_E_DEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cu = prop.multiProcessorCount;
  if (scratch_address(device, &ctx->scratch) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return OPEN_E_DEVICE;
  }
  *out = ctx;
  return OPEN_OK;
}

open_status open_destroy(open_ctx *ctx) {
  if (!ctx) return OPEN_E_INVALID;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < open_ctx::WS_COUNT; ++i)
    if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return OPEN_OK;
}

open_status open_set_stream(open_ctx *ctx, void *hip_stream) {
  if (!ctx) return OPEN_E_INVALID;
  ctx->stream = (hipStream_t)hip_stream;
  return OPEN_OK;
}

const char *open_last_error(const open_ctx *ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

open_status open_profile(open_ctx *ctx, int32_t enable) {
  if (!ctx) return OPEN_E_INVALID;
  ctx->prof_on = enable != 0;
  return OPEN_OK;
}

int32_t open_profile_read(open_ctx *ctx, const char **names, double *total_ms, int64_t *launches, int32_t max,
                          int32_t reset) {
  if (!ctx) return -1;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return -1;
  std::vector<const char *> nm;
  std::vector<double> tot;
  std::vector<int64_t> cnt;
  for (const auto &r : ctx->prof_recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.beg, r.end) != hipSuccess) continue;
    size_t i = 0;
    while (i < nm.size() && strcmp(nm[i], r.name) != 0) ++i;
    if (i == nm.size()) {
      nm.push_back(r.name);
      tot.push_back(0.0);
      cnt.push_back(0);
    }
    tot[i] += ms;
    cnt[i] += 1;
  }
  const int32_t n = (int32_t)nm.size();
  for (int32_t i = 0; i < n && i < max; ++i) {
    if (names) names[i] = nm[i];
    if (total_ms) total_ms[i] = tot[i];
    if (launches) launches[i] = cnt[i];
  }
  if (reset) {
    ctx->prof_recs.clear();
    ctx->prof_pool_used = 0;
  }
  return n;
}

open_status open_sync(open_ctx *ctx) {
  if (!ctx) return OPEN_E_INVALID;
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return OPEN_OK;
}

// Shared front half of open_foldin and open_autotune: validation and bucketing.  Rows can
// reach the split-K length only when F has at least kSplitMin rows (column indices are
// unique within a row); then the total entry count is read back to size its work.
static open_status foldin_prepare(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m,
                                  const int64_t *row_ptr, const int32_t *col, const float *val, float lambda,
                                  float *U_out, RowRef **list, int64_t **cls, int64_t *nnz_split) {
  *nnz_split = -1;
  if (!rank_ok(k)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (n <= 0 || !F) return fail(ctx, OPEN_E_INVALID, "factor matrix must be non-empty");
  if (!(lambda >= 0.0f) || !isfinite(lambda)) return fail(ctx, OPEN_E_INVALID, "lambda must be finite and >= 0");
  open_status st = check_csr(ctx, m, row_ptr, col, val);
  if (st) return st;
  if (m > 0 && !U_out) return fail(ctx, OPEN_E_INVALID, "output must not be NULL");
  if (m == 0) return OPEN_OK;
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (n >= kSplitMin) {
    int64_t *h;
    if ((st = pinned_get(ctx, sizeof(int64_t), (void **)&h))) return st;
    OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    *nnz_split = *h;
  }
  if ((st = bucket_rows(ctx, m, row_ptr, k, list, cls, *nnz_split >= 0 ? kSplitMin : INT64_MAX))) return st;
  return OPEN_OK;
}

open_status open_foldin(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m, const int64_t *row_ptr,
                        const int32_t *col, const float *val, float lambda, int32_t weighted, float *U_out,
                        int32_t *row_status) {
  if (!ctx) return OPEN_E_INVALID;
  RowRef *list = nullptr;
  int64_t *cls = nullptr, nnz = -1;
  open_status st = foldin_prepare(ctx, F, n, k, m, row_ptr, col, val, lambda, U_out, &list, &cls, &nnz);
  if (st || m == 0) return st;
  if ((st = rowsolve_launch(ctx, F, n, k, row_ptr, col, val, lambda, weighted, list, cls, U_out, row_status, m)))
    return st;
  if (nnz >= 0) return splitk_launch(ctx, F, n, k, col, val, lambda, weighted, list, cls, U_out, row_status, m, nnz);
  return OPEN_OK;
}

open_status open_foldin_graph(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m, const int64_t *row_ptr,
                              const int32_t *col, const float *val, float lambda, int32_t weighted, float *U_out,
                              int32_t *row_status) {
  if (!ctx) return OPEN_E_INVALID;
  if (k == 64 || n >= kSplitMin)
    return fail(ctx, OPEN_E_UNSUPPORTED, "graph replay needs rank 8, 16 or 32 and fewer than 1024 factor rows");
  open_ctx::FoldinKey key;
  memset(&key, 0, sizeof(key));
  key.F = F;
  key.n = n;
  key.k = k;
  key.m = m;
  key.row_ptr = row_ptr;
  key.col = col;
  key.val = val;
  key.lambda = lambda;
  key.weighted = weighted;
  key.U = U_out;
  key.status = row_status;
  if (rank_ok(k)) memcpy(key.tune, ctx->tune[rank_index(k)], sizeof(key.tune));
  key.ws_gen = ctx->ws_gen;
  if (ctx->graph_exec && memcmp(&key, &ctx->gkey, sizeof(key)) == 0) {
    OPEN_HIP_TRY(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
    return OPEN_OK;
  }
  // eager pass: validates the arguments, sizes the workspaces and produces this call's result
  open_status st = open_foldin(ctx, F, n, k, m, row_ptr, col, val, lambda, weighted, U_out, row_status);
  if (st || m == 0) return st;
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
  hipGraph_t g;
  st = graph_capture(ctx, [&]() { return open_foldin(ctx, F, n, k, m, row_ptr, col, val, lambda, weighted, U_out,
                                               row_status); }, &g);
  if (st) return st;
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    return fail(ctx, OPEN_E_DEVICE, "graph instantiation failed");
  }
  ctx->graph = g;
  ctx->graph_exec = ex;
  key.ws_gen = ctx->ws_gen;  // the eager pass may have grown a workspace before the recording
  memcpy(&ctx->gkey, &key, sizeof(key));  // byte copy: the key is compared with memcmp
  return OPEN_OK;
}

open_status open_foldin_noalloc(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m,
                                const int64_t *row_ptr, const int32_t *col, const float *val, float lambda,
                                int32_t weighted, float *U_out, int32_t *row_status) {
  if (!ctx) return OPEN_E_INVALID;
  if (!rank_ok(k)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (n <= 0 || !F) return fail(ctx, OPEN_E_INVALID, "factor matrix must be non-empty");
  if (n >= kSplitMin)
    return fail(ctx, OPEN_E_UNSUPPORTED, "the allocation-free fold-in needs fewer than 1024 factor rows");
  if (!(lambda >= 0.0f) || !isfinite(lambda)) return fail(ctx, OPEN_E_INVALID, "lambda must be finite and >= 0");
  open_status st = check_csr(ctx, m, row_ptr, col, val);
  if (st) return st;
  if (m > kNoAllocMaxRows)
    return fail(ctx, OPEN_E_INVALID, "the allocation-free fold-in takes at most " + std::to_string(kNoAllocMaxRows) +
                                         " rows per call (got " + std::to_string(m) + ")");
  if (m > 0 && !U_out) return fail(ctx, OPEN_E_INVALID, "output must not be NULL");
  if (!ctx->scratch) return fail(ctx, OPEN_E_DEVICE, "scratch address unknown");
  if (sizeof(int32_t) * (size_t)bucket_hist_ints(m) > kScrCls - kScrHist)
    return fail(ctx, OPEN_E_INVALID, "row count exceeds the scratch layout");
  if (m == 0) return OPEN_OK;
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  unsigned char *base = (unsigned char *)ctx->scratch;
  RowRef *list = (RowRef *)(base + kScrList);
  int32_t *hist = (int32_t *)(base + kScrHist);
  int64_t *cls = (int64_t *)(base + kScrCls);
  if ((st = bucket_rows_into(ctx, m, row_ptr, k, hist, list, cls, INT64_MAX))) return st;
  return rowsolve_launch(ctx, F, n, k, row_ptr, col, val, lambda, weighted, list, cls, U_out, row_status, m);
}

int64_t open_foldin_noalloc_max_rows(void) { return kNoAllocMaxRows; }

int32_t open_tune_info(int32_t k, const char **names, int32_t *nvar, int32_t max) {
  int ng = 0;
  const ClassGroup *g = class_groups(k, &ng);
  if (!g) return -1;
  for (int i = 0; i < ng && i < max; ++i) {
    if (names) names[i] = g[i].name;
    if (nvar) nvar[i] = g[i].nvar;
  }
  return ng;
}

open_status open_tune_get(open_ctx *ctx, int32_t k, int8_t *choice, int32_t count) {
  if (!ctx) return OPEN_E_INVALID;
  int ng = 0;
  if (!class_groups(k, &ng)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (count != ng || !choice) return fail(ctx, OPEN_E_INVALID, "choice array must hold one entry per class group");
  memcpy(choice, ctx->tune[rank_index(k)], (size_t)ng);
  return OPEN_OK;
}

open_status open_tune_set(open_ctx *ctx, int32_t k, const int8_t *choice, int32_t count) {
  if (!ctx) return OPEN_E_INVALID;
  int ng = 0;
  const ClassGroup *g = class_groups(k, &ng);
  if (!g) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (count != ng || !choice) return fail(ctx, OPEN_E_INVALID, "choice array must hold one entry per class group");
  for (int i = 0; i < ng; ++i)
    if (choice[i] < 0 || choice[i] >= g[i].nvar) return fail(ctx, OPEN_E_INVALID, "variant out of range");
  memcpy(ctx->tune[rank_index(k)], choice, (size_t)ng);
  return OPEN_OK;
}

open_status open_autotune(open_ctx *ctx, const float *F, int32_t n, int32_t k, int64_t m, const int64_t *row_ptr,
                          const int32_t *col, const float *val, float lambda, int32_t weighted, float *U_out,
                          int32_t *row_status, int32_t reps, double *ms_out) {
  if (!ctx) return OPEN_E_INVALID;
  if (reps < 1) return fail(ctx, OPEN_E_INVALID, "reps must be >= 1");
  RowRef *list = nullptr;
  int64_t *cls = nullptr, nnz = -1;
  open_status st = foldin_prepare(ctx, F, n, k, m, row_ptr, col, val, lambda, U_out, &list, &cls, &nnz);
  if (st || m == 0) return st;
  if ((st = rowsolve_autotune(ctx, F, n, k, row_ptr, col, val, lambda, weighted, list, cls, U_out, row_status, m,
                              reps, ms_out)))
    return st;
  if (nnz >= 0) return splitk_launch(ctx, F, n, k, col, val, lambda, weighted, list, cls, U_out, row_status, m, nnz);
  return OPEN_OK;
}

}  // extern "C"
