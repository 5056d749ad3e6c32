// ALS-WR fit support: column view of the CSR (exact stable counting sort), the objective
// reduced in float64 in a fixed order, the observed-entry residual, and the sweep driver.
//
// Column view.  Rows are cut into chunks of kChunkRows rows; one wavefront owns a chunk.
//   pass 1  per-chunk column histogram (LDS counters, exact)
//   scan    exclusive scan of the column-major histogram (column j, then chunk) gives, for
//           every (j, chunk), the position of the chunk's first entry of column j
//   pass 2  the wavefront walks its rows in order; the entries of one row have distinct
//           columns, so its lanes place them without conflicts.  Entries land ordered by
//           column and, within a column, by row.
#include <math.h>
#include <string.h>

#include "common.h"

namespace openk {

constexpr int kChunkRows = 256;
constexpr int kCscWaves = 4;  // wavefronts per block
constexpr int kMaxCols = 4096;

__global__ __launch_bounds__(kCscWaves * 64) void k_csc_count(int64_t m, int n, const int64_t *__restrict__ ptr,
                                                              const int32_t *__restrict__ col, int nchunk,
                                                              int32_t *__restrict__ hist) {
  extern __shared__ int cnt_s[];  // [kCscWaves][n]
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int *cnt = cnt_s + w * n;
  const int64_t chunk = (int64_t)blockIdx.x * kCscWaves + w;
  for (int j = lane; j < n; j += 64) cnt[j] = 0;
  __syncthreads();
  if (chunk < nchunk) {
    const int64_t r0 = chunk * kChunkRows;
    const int64_t r1 = r0 + kChunkRows < m ? r0 + kChunkRows : m;
    for (int64_t t = ptr[r0] + lane; t < ptr[r1]; t += 64) {
      const int j = col[t];
      if (j >= 0 && j < n) atomicAdd(&cnt[j], 1);
    }
  }
  __syncthreads();
  if (chunk < nchunk)
    for (int j = lane; j < n; j += 64) hist[(int64_t)j * nchunk + chunk] = cnt[j];
}

__global__ __launch_bounds__(kCscWaves * 64) void k_csc_place(int64_t m, int n, const int64_t *__restrict__ ptr,
                                                              const int32_t *__restrict__ col,
                                                              const float *__restrict__ val, int nchunk,
                                                              const int64_t *__restrict__ base,
                                                              int32_t *__restrict__ row_idx,
                                                              float *__restrict__ cval) {
  extern __shared__ int64_t pos_s[];  // [kCscWaves][n]
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t *pos = pos_s + (int64_t)w * n;
  const int64_t chunk = (int64_t)blockIdx.x * kCscWaves + w;
  if (chunk >= nchunk) return;
  for (int j = lane; j < n; j += 64) pos[j] = base[(int64_t)j * nchunk + chunk];
  const int64_t r0 = chunk * kChunkRows;
  const int64_t r1 = r0 + kChunkRows < m ? r0 + kChunkRows : m;
  for (int64_t i = r0; i < r1; ++i) {
    for (int64_t t = ptr[i] + lane; t < ptr[i + 1]; t += 64) {
      const int j = col[t];
      if (j < 0 || j >= n) continue;  // rejected by the index check
      const int64_t p = pos[j]++;     // columns are distinct within a row
      row_idx[p] = (int32_t)i;
      cval[p] = val[t];
    }
  }
}

// Exclusive scan of int32 counts into int64 offsets, three phases over blocks of 1024.
__global__ __launch_bounds__(1024) void k_scan_blocks(const int32_t *__restrict__ in, int64_t len,
                                                      int64_t *__restrict__ out, int64_t *__restrict__ block_sum) {
  __shared__ int64_t s[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  s[threadIdx.x] = i < len ? in[i] : 0;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  if (i < len) out[i] = s[threadIdx.x] - (i < len ? in[i] : 0);
  if (threadIdx.x == 1023) block_sum[blockIdx.x] = s[1023];
}

__global__ __launch_bounds__(1024) void k_scan_sums(int64_t *__restrict__ block_sum, int64_t nb) {
  // single block: exclusive scan of nb block sums, sequential chunks per thread
  __shared__ int64_t part[1024];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = threadIdx.x * per;
  const int64_t b1 = b0 + per < nb ? b0 + per : nb;
  int64_t acc = 0;
  for (int64_t i = b0; i < b1; ++i) acc += block_sum[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int64_t i = b0; i < b1; ++i) {
    const int64_t v = block_sum[i];
    block_sum[i] = run;
    run += v;
  }
}

__global__ void k_scan_add(int64_t *__restrict__ out, int64_t len, const int64_t *__restrict__ block_sum) {
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < len) out[i] += block_sum[blockIdx.x];
}

// col_ptr[j] = base[j * nchunk] (first chunk of column j), col_ptr[n] = number of entries
__global__ void k_colptr(const int64_t *__restrict__ base, const int32_t *__restrict__ hist, int n, int nchunk,
                         int64_t *__restrict__ col_ptr) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t len = (int64_t)n * nchunk;
  if (j < n) col_ptr[j] = nchunk > 0 ? base[(int64_t)j * nchunk] : 0;
  if (j == n) col_ptr[n] = len > 0 ? base[len - 1] + hist[len - 1] : 0;
}

// flag[0] |= 1 if some column index lies outside [0, n)
__global__ void k_check_cols(int64_t nnz, const int32_t *__restrict__ col, int n, int *__restrict__ flag) {
  int bad = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * blockDim.x)
    bad |= (col[t] < 0) | (col[t] >= n);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Synchronous check that every column index is in range (OPEN_E_INVALID otherwise).
static open_status check_cols(open_ctx *ctx, int64_t nnz, const int32_t *col, int n) {
  if (nnz <= 0) return OPEN_OK;
  void *flag;
  int *h;
  open_status st;
  if ((st = ws_get(ctx, open_ctx::WS_FLAG, 256, &flag))) return st;
  if ((st = pinned_get(ctx, 64, (void **)&h))) return st;
  OPEN_LAUNCH(ctx, "fill", k_fill_i32, dim3(1), dim3(64), 0, (int *)flag, 1, 0);
  int64_t blocks = (nnz + 255) / 256;
  if (blocks > ctx->num_cu * 8) blocks = ctx->num_cu * 8;
  OPEN_LAUNCH(ctx, "check_cols", k_check_cols, dim3((unsigned)blocks), dim3(256), 0, nnz, col, n, (int *)flag);
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (h[0]) return fail(ctx, OPEN_E_INVALID, "a column index lies outside [0, n)");
  return OPEN_OK;
}

open_status csr_to_csc_dev(open_ctx *ctx, int64_t m, int n, const int64_t *row_ptr, const int32_t *col,
                                   const float *val, int64_t *col_ptr, int32_t *row_idx, float *cval) {
  const int nchunk = (int)((m + kChunkRows - 1) / kChunkRows);
  const int64_t len = (int64_t)n * nchunk;
  const int64_t nb = (len + 1023) / 1024;
  void *hist, *base, *bsum;
  open_status st;
  if ((st = ws_get(ctx, open_ctx::WS_HIST, sizeof(int32_t) * (size_t)(len > 0 ? len : 1), &hist))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_SPLIT, sizeof(int64_t) * (size_t)(len > 0 ? len : 1), &base))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_RED, sizeof(int64_t) * (size_t)(nb > 0 ? nb : 1), &bsum))) return st;
  const int blocks = (nchunk + kCscWaves - 1) / kCscWaves;
  if (nchunk > 0) {
    OPEN_LAUNCH(ctx, "csc_count", k_csc_count, dim3(blocks), dim3(kCscWaves * 64), sizeof(int) * kCscWaves * n, m, n,
                row_ptr, col, nchunk, (int32_t *)hist);
    OPEN_LAUNCH(ctx, "scan_blocks", k_scan_blocks, dim3((unsigned)nb), dim3(1024), 0, (const int32_t *)hist, len,
                (int64_t *)base, (int64_t *)bsum);
    OPEN_LAUNCH(ctx, "scan_sums", k_scan_sums, dim3(1), dim3(1024), 0, (int64_t *)bsum, nb);
    OPEN_LAUNCH(ctx, "scan_add", k_scan_add, dim3((unsigned)nb), dim3(1024), 0, (int64_t *)base, len,
                (const int64_t *)bsum);
  }
  OPEN_LAUNCH(ctx, "csc_colptr", k_colptr, dim3((n + 1 + 255) / 256), dim3(256), 0, (const int64_t *)base,
              (const int32_t *)hist, n, nchunk, col_ptr);
  if (nchunk > 0) {
    OPEN_LAUNCH(ctx, "csc_place", k_csc_place, dim3(blocks), dim3(kCscWaves * 64), sizeof(int64_t) * kCscWaves * n, m,
                n, row_ptr, col, val, nchunk, (const int64_t *)base, row_idx, cval);
  }
  return OPEN_OK;
}

// ---------------------------------------------------------------- objective and residual
constexpr int kRedBlocks = 1024;

// One wavefront per row (grid-stride).  Per row the squared errors and |u_i|^2 are formed
// in float32 and added to a per-lane float64 accumulator; lanes and waves are combined in
// a fixed order, then a second kernel adds the block partials in order.
template <int K>
__global__ __launch_bounds__(256) void k_objective_rows(int64_t m, int n, const int64_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ col,
                                                        const float *__restrict__ val, const float *__restrict__ U,
                                                        const float *__restrict__ V, float lambda, int weighted,
                                                        double *__restrict__ part) {
  __shared__ double red[256];
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < m; i += nw) {
    const float *u = U + i * K;
    const int64_t b = ptr[i], e = ptr[i + 1];
    for (int64_t t = b + lane; t < e; t += 64) {
      const int j = col[t];
      if (j < 0 || j >= n) continue;
      const float *v = V + (int64_t)j * K;
      float p = 0.f;
#pragma unroll
      for (int a = 0; a < K; ++a) p = __builtin_fmaf(u[a], v[a], p);
      const float d = val[t] - p;
      acc += (double)(d * d);
    }
    if (lane < K) {
      const float w = weighted ? (float)(e - b) : 1.0f;
      acc += (double)lambda * (double)w * (double)(u[lane] * u[lane]);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// lambda * sum_j w^j |v_j|^2 with w^j from the column pointer (or 1); one block, fixed order
template <int K>
__global__ __launch_bounds__(256) void k_objective_cols(int n, const int64_t *__restrict__ col_ptr,
                                                        const float *__restrict__ V, float lambda, int weighted,
                                                        const double *__restrict__ part, int nparts,
                                                        double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < K; ++a) s = __builtin_fmaf(V[(int64_t)j * K + a], V[(int64_t)j * K + a], s);
    const double w = weighted ? (double)(col_ptr[j + 1] - col_ptr[j]) : 1.0;
    acc += (double)lambda * w * (double)s;
  }
  for (int b = threadIdx.x; b < nparts; b += 256) acc += part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <int K>
__global__ __launch_bounds__(256) void k_residual(int64_t m, int n, const int64_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col, const float *__restrict__ val,
                                                  const float *__restrict__ U, const float *__restrict__ V,
                                                  float *__restrict__ rho) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < m; i += nw) {
    const float *u = U + i * K;
    const int64_t b = ptr[i], e = ptr[i + 1];
    float acc = 0.f;
    for (int64_t t = b + lane; t < e; t += 64) {
      const int j = col[t];
      if (j < 0 || j >= n) continue;
      const float *v = V + (int64_t)j * K;
      float p = 0.f;
#pragma unroll
      for (int a = 0; a < K; ++a) p = __builtin_fmaf(u[a], v[a], p);
      const float d = val[t] - p;
      acc = __builtin_fmaf(d, d, acc);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) rho[i] = e > b ? sqrtf(acc / (float)(e - b)) : 0.f;
  }
}

template <int K>
static open_status objective_impl(open_ctx *ctx, int64_t m, int n, const int64_t *row_ptr, const int32_t *col,
                                  const float *val, const float *U, const float *V, float lambda, int weighted,
                                  const int64_t *col_ptr, double *out_dev) {
  void *part;
  open_status st;
  if ((st = ws_get(ctx, open_ctx::WS_MISC, sizeof(double) * (kRedBlocks + 8), &part))) return st;
  OPEN_LAUNCH(ctx, "objective_rows", k_objective_rows<K>, dim3(kRedBlocks), dim3(256), 0, m, n, row_ptr, col, val, U, V,
              lambda, weighted, (double *)part);
  OPEN_LAUNCH(ctx, "objective_cols", k_objective_cols<K>, dim3(1), dim3(256), 0, n, col_ptr, V, lambda, weighted,
              (const double *)part, kRedBlocks, out_dev);
  return OPEN_OK;
}

static open_status objective_dispatch(open_ctx *ctx, int k, int64_t m, int n, const int64_t *row_ptr,
                                      const int32_t *col, const float *val, const float *U, const float *V,
                                      float lambda, int weighted, const int64_t *col_ptr, double *out_dev) {
  switch (k) {
    case 8: return objective_impl<8>(ctx, m, n, row_ptr, col, val, U, V, lambda, weighted, col_ptr, out_dev);
    case 16: return objective_impl<16>(ctx, m, n, row_ptr, col, val, U, V, lambda, weighted, col_ptr, out_dev);
    case 32: return objective_impl<32>(ctx, m, n, row_ptr, col, val, U, V, lambda, weighted, col_ptr, out_dev);
    default: return objective_impl<64>(ctx, m, n, row_ptr, col, val, U, V, lambda, weighted, col_ptr, out_dev);
  }
}

}  // namespace openk

using namespace openk;

extern "C" {

open_status open_csr_to_csc(open_ctx *ctx, int64_t m, int32_t n, const int64_t *row_ptr, const int32_t *col,
                            const float *val, int64_t *col_ptr, int32_t *row_idx, float *cval) {
  if (!ctx) return OPEN_E_INVALID;
  if (m < 0 || m >= INT32_MAX) return fail(ctx, OPEN_E_INVALID, "row count must be in [0, 2^31 - 1)");
  if (n <= 0 || n > kMaxCols) return fail(ctx, OPEN_E_INVALID, "column count must be in [1, 4096]");
  if (!row_ptr || !col_ptr || (m > 0 && (!col || !val || !row_idx || !cval)))
    return fail(ctx, OPEN_E_INVALID, "pointers must not be NULL");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int64_t nnz = 0;
  if (m > 0) {
    OPEN_HIP_TRY(ctx, hipMemcpyAsync(&nnz, row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  open_status st = check_cols(ctx, nnz, col, n);
  if (st) return st;
  return csr_to_csc_dev(ctx, m, n, row_ptr, col, val, col_ptr, row_idx, cval);
}

open_status open_objective(open_ctx *ctx, int64_t m, int32_t n, int32_t k, const int64_t *row_ptr,
                           const int32_t *col, const float *val, const float *U, const float *V, float lambda,
                           int32_t weighted, double *out) {
  if (!ctx) return OPEN_E_INVALID;
  if (!(k == 8 || k == 16 || k == 32 || k == 64)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (m < 0 || m >= INT32_MAX || n <= 0 || n > kMaxCols || !out || !U || !V || !row_ptr)
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  // the column weights w^j are the column counts: they come from the column-view pass
  void *cp, *ri, *cv;
  open_status st;
  int64_t nnz;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(&nnz, row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if ((st = check_cols(ctx, nnz, col, n))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_CSC_PTR, sizeof(int64_t) * (n + 1), &cp))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_CSC_IDX, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1), &ri))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_CSC_VAL, sizeof(float) * (size_t)(nnz > 0 ? nnz : 1), &cv))) return st;
  if ((st = csr_to_csc_dev(ctx, m, n, row_ptr, col, val, (int64_t *)cp, (int32_t *)ri, (float *)cv))) return st;
  double *h;
  if ((st = pinned_get(ctx, 64, (void **)&h))) return st;
  void *d;
  if ((st = ws_get(ctx, open_ctx::WS_OBJ, 256, &d))) return st;
  if ((st = objective_dispatch(ctx, k, m, n, row_ptr, col, val, U, V, lambda, weighted, (const int64_t *)cp,
                               (double *)d)))
    return st;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out = h[0];
  return OPEN_OK;
}

open_status open_residual(open_ctx *ctx, int64_t m, int32_t n, int32_t k, const int64_t *row_ptr,
                          const int32_t *col, const float *val, const float *U, const float *V, float *rho) {
  if (!ctx) return OPEN_E_INVALID;
  if (!(k == 8 || k == 16 || k == 32 || k == 64)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (m < 0 || m >= INT32_MAX || n <= 0 || (m > 0 && (!rho || !U || !V || !row_ptr)))
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  if (m == 0) return OPEN_OK;
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int64_t blocks = (m + 3) / 4;
  if (blocks > ctx->num_cu * 8) blocks = ctx->num_cu * 8;
  const dim3 g((unsigned)blocks), b(256);
  switch (k) {
    case 8: OPEN_LAUNCH(ctx, "residual", k_residual<8>, g, b, 0, m, n, row_ptr, col, val, U, V, rho); break;
    case 16: OPEN_LAUNCH(ctx, "residual", k_residual<16>, g, b, 0, m, n, row_ptr, col, val, U, V, rho); break;
    case 32: OPEN_LAUNCH(ctx, "residual", k_residual<32>, g, b, 0, m, n, row_ptr, col, val, U, V, rho); break;
    default: OPEN_LAUNCH(ctx, "residual", k_residual<64>, g, b, 0, m, n, row_ptr, col, val, U, V, rho); break;
  }
  return OPEN_OK;
}

// ALS-WR sweeps.  The column view and both bucketings are built once per call.
open_status open_fit(open_ctx *ctx, int64_t m, int32_t n, int32_t k, const int64_t *row_ptr, const int32_t *col,
                     const float *val, float lambda, int32_t weighted, int32_t sweeps, float *U, float *V,
                     double *obj_hist) {
  if (!ctx) return OPEN_E_INVALID;
  if (!(k == 8 || k == 16 || k == 32 || k == 64)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (m <= 0 || m >= INT32_MAX || n <= 0 || n > kMaxCols || sweeps < 0 || !row_ptr || !col || !val || !U || !V)
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  if (!(lambda >= 0.0f) || !isfinite(lambda)) return fail(ctx, OPEN_E_INVALID, "lambda must be finite and >= 0");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  int64_t nnz;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(&nnz, row_ptr + m, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  // caller-independent buffers of this call: the column view and the two bucketings
  int64_t *cp = nullptr;
  int32_t *ri = nullptr;
  RowRef *list_r = nullptr, *list_c = nullptr;
  float *cv = nullptr;
  int64_t *cls_r = nullptr, *cls_c = nullptr;
  double *obj_d = nullptr;
  open_status st = OPEN_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(cp);
    (void)hipFree(ri);
    (void)hipFree(cv);
    (void)hipFree(list_r);
    (void)hipFree(list_c);
    (void)hipFree(cls_r);
    (void)hipFree(cls_c);
    (void)hipFree(obj_d);
  };
  if (hipMalloc(&cp, sizeof(int64_t) * (n + 1)) != hipSuccess ||
      hipMalloc(&ri, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)) != hipSuccess ||
      hipMalloc(&cv, sizeof(float) * (size_t)(nnz > 0 ? nnz : 1)) != hipSuccess ||
      hipMalloc(&list_r, sizeof(RowRef) * (size_t)m) != hipSuccess ||
      hipMalloc(&list_c, sizeof(RowRef) * (size_t)n) != hipSuccess ||
      hipMalloc(&cls_r, sizeof(int64_t) * 2 * kNumClasses) != hipSuccess ||
      hipMalloc(&cls_c, sizeof(int64_t) * 2 * kNumClasses) != hipSuccess ||
      hipMalloc(&obj_d, sizeof(double) * 2 * (sweeps > 0 ? sweeps : 1)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(ctx, OPEN_E_NOMEM, "fit buffers");
  }
  do {
    if ((st = check_cols(ctx, nnz, col, n))) break;
    if ((st = csr_to_csc_dev(ctx, m, n, row_ptr, col, val, cp, ri, cv))) break;
    RowRef *l;
    int64_t *c;
    if ((st = bucket_rows(ctx, m, row_ptr, k, &l, &c, kSplitMin))) break;
    if (hipMemcpyAsync(list_r, l, sizeof(RowRef) * m, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(cls_r, c, sizeof(int64_t) * 2 * kNumClasses, hipMemcpyDeviceToDevice, ctx->stream) !=
            hipSuccess) {
      st = fail(ctx, OPEN_E_DEVICE, "copy");
      break;
    }
    if ((st = bucket_rows(ctx, n, cp, k, &l, &c, kSplitMin))) break;
    if (hipMemcpyAsync(list_c, l, sizeof(RowRef) * n, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(cls_c, c, sizeof(int64_t) * 2 * kNumClasses, hipMemcpyDeviceToDevice, ctx->stream) !=
            hipSuccess) {
      st = fail(ctx, OPEN_E_DEVICE, "copy");
      break;
    }
    auto sweep = [&]() -> open_status {
      open_status e;
      if ((e = rowsolve_launch(ctx, V, n, k, row_ptr, col, val, lambda, weighted, list_r, cls_r, U, nullptr, m)))
        return e;
      if ((e = splitk_launch(ctx, V, n, k, col, val, lambda, weighted, list_r, cls_r, U, nullptr, m, nnz))) return e;
      if ((e = rowsolve_launch(ctx, U, (int)m, k, cp, ri, cv, lambda, weighted, list_c, cls_c, V, nullptr, n)))
        return e;
      return splitk_launch(ctx, U, (int)m, k, ri, cv, lambda, weighted, list_c, cls_c, V, nullptr, n, nnz);
    };
    if (!obj_hist && sweeps >= 2 && !ctx->prof_on) {
      // the first sweep runs eagerly (and sizes the workspaces); the others replay it as one graph
      if ((st = sweep())) break;
      hipGraph_t g = nullptr;
      if ((st = graph_capture(ctx, sweep, &g))) break;
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(g);
        st = fail(ctx, OPEN_E_DEVICE, "graph instantiation failed");
        break;
      }
      for (int s = 1; s < sweeps && !st; ++s)
        if (hipGraphLaunch(ex, ctx->stream) != hipSuccess) st = fail(ctx, OPEN_E_DEVICE, "graph launch failed");
      (void)hipStreamSynchronize(ctx->stream);  // the graph is released below
      (void)hipGraphExecDestroy(ex);
      (void)hipGraphDestroy(g);
      break;
    }
    for (int s = 0; s < sweeps && !st; ++s) {
      if ((st = rowsolve_launch(ctx, V, n, k, row_ptr, col, val, lambda, weighted, list_r, cls_r, U, nullptr, m)))
        break;
      if ((st = splitk_launch(ctx, V, n, k, col, val, lambda, weighted, list_r, cls_r, U, nullptr, m, nnz))) break;
      if (obj_hist &&
          (st = objective_dispatch(ctx, k, m, n, row_ptr, col, val, U, V, lambda, weighted, cp, obj_d + 2 * s)))
        break;
      if ((st = rowsolve_launch(ctx, U, (int)m, k, cp, ri, cv, lambda, weighted, list_c, cls_c, V, nullptr, n)))
        break;
      if ((st = splitk_launch(ctx, U, (int)m, k, ri, cv, lambda, weighted, list_c, cls_c, V, nullptr, n, nnz))) break;
      if (obj_hist &&
          (st = objective_dispatch(ctx, k, m, n, row_ptr, col, val, U, V, lambda, weighted, cp, obj_d + 2 * s + 1)))
        break;
    }
    if (!st && obj_hist && sweeps > 0) {
      if (hipMemcpyAsync(obj_hist, obj_d, sizeof(double) * 2 * sweeps, hipMemcpyDeviceToHost, ctx->stream) ||
          hipStreamSynchronize(ctx->stream))
        st = fail(ctx, OPEN_E_DEVICE, "objective copy");
    }
  } while (0);
  cleanup();
  return st;
}

// Warm-started refit on the union of the offline rows and newly arrived rows: the new rows are
// folded in against the current V, then `sweeps` ALS sweeps run on the union from there.
open_status open_refit(open_ctx *ctx, int64_t m_old, int64_t m_new, int32_t n, int32_t k, const int64_t *row_ptr,
                       const int32_t *col, const float *val, float lambda, int32_t weighted, int32_t sweeps, float *U,
                       float *V, double *obj_hist) {
  if (!ctx) return OPEN_E_INVALID;
  if (m_old < 0 || m_new < 0 || m_old + m_new <= 0 || !U || !V || !row_ptr)
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  open_status st;
  if (m_new > 0 &&
      (st = open_foldin(ctx, V, n, k, m_new, row_ptr + m_old, col, val, lambda, weighted, U + m_old * (int64_t)k,
                        nullptr)))
    return st;
  return open_fit(ctx, m_old + m_new, n, k, row_ptr, col, val, lambda, weighted, sweeps, U, V, obj_hist);
}

}  // extern "C"
