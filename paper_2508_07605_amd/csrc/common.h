// Internal helpers shared by the HIP sources of libopen (device intrinsics, launch checks,
// the context structure).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/open.h"

namespace openk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16 __attribute__((ext_vector_type(16)));

constexpr int kWave = 64;

// ---------------------------------------------------------------- quad (4-lane) exchange
// DPP quad_perm: every lane of a quad reads lane `src` of its own quad.
__device__ __forceinline__ float quad_bcast(float x, int src) {
  switch (src) {
    case 0: return __builtin_amdgcn_update_dpp(0.0f, x, 0x00, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_update_dpp(0.0f, x, 0x55, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_update_dpp(0.0f, x, 0xaa, 0xf, 0xf, false);
    default: return __builtin_amdgcn_update_dpp(0.0f, x, 0xff, 0xf, 0xf, false);
  }
}
template <int SRC>
__device__ __forceinline__ float quad_bcast_c(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), SRC * 0x55, 0xf, 0xf, true));
}
// partner lane q^1 and q^2 within the quad
__device__ __forceinline__ float quad_xor1(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xb1, 0xf, 0xf, true));
}
__device__ __forceinline__ float quad_xor2(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x4e, 0xf, 0xf, true));
}
__device__ __forceinline__ int quad_xor1_i(int x) { return __builtin_amdgcn_mov_dpp(x, 0xb1, 0xf, 0xf, true); }
__device__ __forceinline__ int quad_xor2_i(int x) { return __builtin_amdgcn_mov_dpp(x, 0x4e, 0xf, 0xf, true); }

// ---------------------------------------------------------------- bounds-checked loads
// Raw buffer loads: an offset at or beyond the buffer's byte size (negative offsets wrap to
// large unsigned values) returns zero instead of touching memory, so padded and invalid
// entries need no branch.  Word 3 is the gfx9-family raw-buffer format.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint64_t bytes) {
  const int nrec = bytes >= 0xffffffffull ? (int)0xffffffff : (int)(uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, nrec, 0x00020000);
}
__device__ __forceinline__ float bload_f32(__amdgpu_buffer_rsrc_t r, int off_bytes) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off_bytes, 0, 0));
}
__device__ __forceinline__ int bload_i32(__amdgpu_buffer_rsrc_t r, int off_bytes) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, off_bytes, 0, 0);
}
// Value of x in lane `l` (a wave-uniform lane).  The builtin takes and returns int, so a
// float goes through its bits: passed as a float it would be converted to an integer value.
__device__ __forceinline__ float readlane_f32(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ f4 bload_f4(__amdgpu_buffer_rsrc_t r, int off_bytes) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off_bytes, 0, 0));
}

// 16 independent 4x4 outer products: lanes 4b..4b+3 form block b; block b accumulates
// D_b[i][j] += A_b[i] * B_b[j] with A_b[i] from lane 4b+i and B_b[j] from lane 4b+j.
// Result layout: lane 4b+j holds column j of block b, register v = row v.
__device__ __forceinline__ f4 mfma4x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// lane l's value of a 64-bit per-lane quantity (l wave-uniform)
__device__ __forceinline__ int64_t readlane_i64(int64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    int y = __shfl_xor(x, off, kWave);
    x = x > y ? x : y;
  }
  return x;
}

// fill an int32 array with a value (used instead of memset so the work can sit in a graph)
__global__ void k_fill_i32(int *p, int64_t n, int v);

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // tile (i >= j)

// Compile-time loop: f(std::integral_constant<int, i>) for i = B .. E-1 (E > B), or descending
// for sfor_down<B, E>: i = E-1 .. B.  Indices are constants at the source level, so they can
// select registers and DPP controls.
template <int B, int E, class Fn>
__device__ __forceinline__ void sfor(Fn &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}
template <int B, int E, class Fn>
__device__ __forceinline__ void sfor_down(Fn &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>{});
    sfor_down<B, E - 1>(f);
  }
}

}  // namespace openk

// ---------------------------------------------------------------- context
struct open_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  std::string err;
  // grow-only device workspaces, indexed by purpose
  enum {
    WS_HIST, WS_CLS, WS_LIST, WS_CSC_PTR, WS_CSC_IDX, WS_CSC_VAL, WS_RED, WS_SPLIT, WS_MISC, WS_FLAG, WS_OBJ,
    WS_PRED, WS_SPLIT_START, WS_SPLIT_PART, WS_SPLIT_FLAG, WS_NCF, WS_COUNT
  };
  void *ws[WS_COUNT] = {};
  size_t ws_bytes[WS_COUNT] = {};
  // bumped whenever a workspace is reallocated: a recorded graph holds the old addresses
  uint64_t ws_gen = 0;
  // this device's copy of the library's static scratch array (allocation-free fold-in)
  void *scratch = nullptr;
  // chosen kernel variant of each size-class group, per rank (8, 16, 32, 64); 0 = default
  int8_t tune[4][16] = {};
  // graph capture: while capturing, launches go to cap_stream and nothing may allocate or sync
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  // the fold-in graph of the last open_foldin_graph arguments
  struct FoldinKey {
    const float *F;
    int n, k;
    int64_t m;
    const int64_t *row_ptr;
    const int32_t *col;
    const float *val;
    float lambda;
    int weighted;
    float *U;
    int32_t *status;
    int8_t tune[16];
    uint64_t ws_gen;  // the workspace addresses the recording refers to
  } gkey = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  void *host_pinned = nullptr;  // small pinned staging buffer for synchronous scalar results
  size_t host_pinned_bytes = 0;
  // optional per-kernel timing (HIP events around each launch)
  bool prof_on = false;
  struct ProfRec {
    const char *name;
    hipEvent_t beg, end;
  };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_pool_used = 0;
};

namespace openk {

// set the error message and return the status
inline open_status fail(open_ctx *ctx, open_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

#define OPEN_HIP_TRY(ctx, expr)                                                             \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return ::openk::fail((ctx), OPEN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define OPEN_LAUNCH_CHECK(ctx)                                                              \
  do {                                                                                      \
    hipError_t _e = hipGetLastError();                                                      \
    if (_e != hipSuccess)                                                                   \
      return ::openk::fail((ctx), OPEN_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(_e)); \
  } while (0)

// Kernel launch on the context's stream, timed with events when profiling is on.
void prof_begin(open_ctx *ctx, const char *name);
void prof_end(open_ctx *ctx);
#define OPEN_LAUNCH(ctx, name, kernel, grid, block, shmem, ...)                          \
  do {                                                                                   \
    ::openk::prof_begin((ctx), (name));                                                  \
    hipLaunchKernelGGL(kernel, grid, block, shmem, (ctx)->stream, __VA_ARGS__);          \
    ::openk::prof_end(ctx);                                                              \
    OPEN_LAUNCH_CHECK(ctx);                                                              \
  } while (0)

// device workspace of at least `bytes` for slot `slot` (grows, never shrinks)
open_status ws_get(open_ctx *ctx, int slot, size_t bytes, void **out);
open_status pinned_get(open_ctx *ctx, size_t bytes, void **out);

// Entry of the bucketed row list: the row and its observed range, so a solver reads one
// 16-byte record instead of the list and then the row pointer.
struct RowRef {
  int32_t row, cnt;
  int64_t beg;
};

// ---- internal launchers (defined in the .hip files)
// Row classification + stable counting sort; fills list[m] (row ids grouped by class) and
// cls[2*kNumClasses] = {start, count} per class, on the device.
constexpr int kNumClasses = 17;
constexpr int kSplitClass = 16;  // rows solved by the split-K path
constexpr int64_t kSplitMin = 1024;  // observations from which a row takes the split-K path
open_status bucket_rows(open_ctx *ctx, int64_t m, const int64_t *row_ptr, int k, RowRef **list, int64_t **cls,
                        int64_t split_min, const uint8_t *mask = nullptr);
// The same into caller-provided buffers: hist of bucket_hist_ints(m) ints, list of m entries,
// cls of 2 * kNumClasses.  Every element that is read is written first (no clearing needed).
open_status bucket_rows_into(open_ctx *ctx, int64_t m, const int64_t *row_ptr, int k, int32_t *hist, RowRef *list,
                             int64_t *cls, int64_t split_min, const uint8_t *mask = nullptr);
int64_t bucket_hist_ints(int64_t m);
// rows per block of the bucketing kernels (the per-block class counts are kNumClasses ints)
constexpr int kBucketRowsPerBlock = 2048;
// Column view on the device (stable counting sort); entries with a column outside [0, n) are dropped.
open_status csr_to_csc_dev(open_ctx *ctx, int64_t m, int n, const int64_t *row_ptr, const int32_t *col,
                           const float *val, int64_t *col_ptr, int32_t *row_idx, float *cval);
// Ridge solve of all rows given a bucketing.
open_status rowsolve_launch(open_ctx *ctx, const float *F, int n, int k, const int64_t *row_ptr, const int32_t *col,
                            const float *val, float lambda, int weighted, const RowRef *list, const int64_t *cls,
                            float *X, int32_t *status, int64_t m);
// Split-K solve of the rows of class kSplitClass (F has nF rows, nnz bounds the work).
open_status splitk_launch(open_ctx *ctx, const float *F, int nF, int k, const int32_t *idx, const float *val,
                          float lambda, int weighted, const RowRef *list, const int64_t *cls, float *X,
                          int32_t *status, int64_t m, int64_t nnz);
// Record the launches of fn() into a HIP graph on the context's capture stream (nothing runs;
// allocation and host read-back fail while capturing).
open_status graph_capture(open_ctx *ctx, const std::function<open_status()> &fn, hipGraph_t *out);
// Kernel variants: at most kMaxVariants per class group; rank_index maps 8/16/32/64 to 0..3.
constexpr int kMaxVariants = 4;
int rank_index(int k);
// Time the variants of each populated class group on this batch and keep the fastest;
// ms_out (host, optional) receives [group][kMaxVariants] milliseconds per launch, -1 if untimed.
open_status rowsolve_autotune(open_ctx *ctx, const float *F, int n, int k, const int64_t *row_ptr,
                              const int32_t *col, const float *val, float lambda, int weighted, const RowRef *list,
                              const int64_t *cls, float *X, int32_t *status, int64_t m, int reps, double *ms_out);

}  // namespace openk
