// Row bucketing for the batched ridge solves (fold-in, ALS half-sweeps).
//
// Every row is put in a size class by its observed count n_i, and the row ids are
// written class by class (ascending within a class) by a stable counting sort:
//   class 0              empty rows
//   classes 1..8         dual form, system dimension padded to 4*class (n_i <= min(k, 32))
//   classes 9..15        primal form (k x k system), n_i in (k 2^p, k 2^(p+1)], p = class - 9
//                        (class 9 also takes n_i in (32, 64] at rank 64)
//   class 16             rows long enough for the split-K path
// Exact integer work; the resulting list is independent of scheduling.
#include "common.h"

namespace openk {

__global__ void k_fill_i32(int *p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

constexpr int kRowsPerBlock = kBucketRowsPerBlock;
constexpr int kBucketThreads = 512;
constexpr int kRowsPerWave = kRowsPerBlock / (kBucketThreads / kWave);  // contiguous rows of one wave
// Up to this many blocks the place kernel derives its own offsets from the raw histogram
// (each block reads kNumClasses * nblk counts from L2), so no scan launch is needed.
constexpr int kSelfScanMaxBlocks = 512;

__device__ __forceinline__ int row_class(int64_t cnt, int k, int64_t split_min) {
  if (cnt <= 0) return 0;
  const int dmax = k < 32 ? k : 32;
  if (cnt <= dmax) return (int)((cnt + 3) >> 2);
  if (cnt >= split_min) return kSplitClass;
  // primal: class 9 + floor(log2((n_i - 1) / k)), at least 9 (rank 64 reaches here from
  // n_i = 33, where (n_i - 1) / k is still 0)
  const int64_t r = (cnt - 1) / k;
  int p = r > 0 ? 63 - __clzll((unsigned long long)r) : 0;
  p = p > 6 ? 6 : p;
  return 9 + p;
}

// mask (nullable): rows with mask[i] == 0 are left out of every class (class -1)
constexpr int kPasses = kRowsPerWave / kWave;

// The rows of one wave (kPasses rows per lane, rows wbase + 64 p + lane): all row-pointer
// loads are issued before any is used, so the latency is paid once rather than per pass.
// They go through buffer resources over the wave's rows (nothing past the last row is read),
// so no branch surrounds them.
struct WaveRows {
  int c[kPasses];
  int64_t beg[kPasses];
  int cnt[kPasses];
  int64_t end[kPasses];  // one past the row's last entry (while loading)
  int keep[kPasses];     // row exists and is not masked out (while loading)
};
// issues the loads only; wave_rows_classify uses them
__device__ __forceinline__ void wave_rows_issue(WaveRows &r, int64_t m, const int64_t *__restrict__ ptr,
                                                const uint8_t *__restrict__ mask, int64_t wbase, int lane) {
  // wbase is the same in every lane; as a scalar it keeps the resources in scalar registers
  const int64_t wb = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)((uint64_t)wbase >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wbase));
  const int64_t left = m > wb ? m - wb : 0;
  const int nr = (int)(left < kRowsPerWave ? left : kRowsPerWave);  // rows of the wave that exist
  // first and one-past-last entry of each row through two resources with exact bounds (one
  // 8-byte load each, none straddling a bound)
  const int64_t *pb = ptr + (nr > 0 ? wb : 0);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(pb, (uint64_t)nr * 8), re = make_rsrc(pb + 1, (uint64_t)nr * 8);
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int o = p * kWave + lane;
    r.beg[p] = __builtin_bit_cast(int64_t, __builtin_amdgcn_raw_buffer_load_b64(rb, o * 8, 0, 0));
    r.end[p] = __builtin_bit_cast(int64_t, __builtin_amdgcn_raw_buffer_load_b64(re, o * 8, 0, 0));
  }
  if (mask) {
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(mask + (nr > 0 ? wb : 0), (uint64_t)nr);
#pragma unroll
    for (int p = 0; p < kPasses; ++p) r.keep[p] = __builtin_amdgcn_raw_buffer_load_b8(rm, p * kWave + lane, 0, 0);
  } else {
#pragma unroll
    for (int p = 0; p < kPasses; ++p) r.keep[p] = p * kWave + lane < nr;
  }
}
__device__ __forceinline__ void wave_rows_classify(WaveRows &r, int k, int64_t split_min) {
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int64_t n = r.end[p] - r.beg[p];
    r.cnt[p] = (int)n;
    r.c[p] = r.keep[p] ? row_class(n, k, split_min) : -1;
  }
}
__device__ __forceinline__ void load_wave_rows(WaveRows &r, int64_t m, const int64_t *__restrict__ ptr,
                                               const uint8_t *__restrict__ mask, int k, int64_t split_min,
                                               int64_t wbase, int lane) {
  wave_rows_issue(r, m, ptr, mask, wbase, lane);
  wave_rows_classify(r, k, split_min);
}

// the classes that occur among the wave's rows, as a bit set (the same value in every lane)
__device__ __forceinline__ unsigned wave_classes_present(const WaveRows &r) {
  unsigned bits = 0;
#pragma unroll
  for (int p = 0; p < kPasses; ++p) bits |= r.c[p] >= 0 ? (1u << r.c[p]) : 0u;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) bits |= (unsigned)__shfl_xor((int)bits, off, kWave);
  return (unsigned)__builtin_amdgcn_readfirstlane((int)bits);
}

// per-class count of the wave's rows, class cc held by lane cc; one ballot per pass and
// class present (a fold-in batch has a handful of classes out of 17)
__device__ __forceinline__ int wave_class_counts(const WaveRows &r, int lane, unsigned present) {
  int mine = 0;
#pragma unroll
  for (int p = 0; p < kPasses; ++p)
    for (unsigned b = present; b; b &= b - 1) {
      const int cc = __builtin_ctz(b);
      const int n = __popcll(__ballot(r.c[p] == cc));
      mine += lane == cc ? n : 0;
    }
  return mine;
}

__global__ __launch_bounds__(kBucketThreads) void k_class_count(int64_t m, const int64_t *__restrict__ ptr,
                                                                const uint8_t *__restrict__ mask, int k,
                                                                int64_t split_min, int32_t *__restrict__ hist) {
  __shared__ int h[kNumClasses];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x < kNumClasses) h[threadIdx.x] = 0;
  __syncthreads();
  WaveRows r;
  load_wave_rows(r, m, ptr, mask, k, split_min, (int64_t)blockIdx.x * kRowsPerBlock + (int64_t)w * kRowsPerWave,
                 lane);
  const int mine = wave_class_counts(r, lane, wave_classes_present(r));
  if (lane < kNumClasses) atomicAdd(&h[lane], mine);
  __syncthreads();
  if (threadIdx.x < kNumClasses) hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the class-major histogram (one block); cls[2c] = start, cls[2c+1] = count.
// Each thread owns a contiguous run of up to 32 entries, loaded at once.
__global__ __launch_bounds__(1024) void k_class_scan(int32_t *__restrict__ hist, int nblk,
                                                     int64_t *__restrict__ cls) {
  __shared__ int64_t part[1024];
  const int total = kNumClasses * nblk;
  const int per = (total + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  const int b1 = b0 + per < total ? b0 + per : total;
  constexpr int R = 32;
  int v[R];
  int64_t s = 0;
  if (per <= R) {
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = b0 + u < b1 ? hist[b0 + u] : 0;
#pragma unroll
    for (int u = 0; u < R; ++u) s += v[u];
  } else {
    for (int i = b0; i < b1; ++i) s += hist[i];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  const int64_t total_rows = part[1023];
  int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  if (per <= R) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (b0 + u < b1) hist[b0 + u] = (int32_t)run;
      run += v[u];
    }
  } else {
    for (int i = b0; i < b1; ++i) {
      const int64_t h = hist[i];
      hist[i] = (int32_t)run;
      run += h;
    }
  }
  __syncthreads();
  if (threadIdx.x < kNumClasses) {
    const int c = threadIdx.x;
    const int64_t start = nblk > 0 ? (int64_t)hist[(int64_t)c * nblk] : 0;
    const int64_t end = c + 1 < kNumClasses && nblk > 0 ? (int64_t)hist[(int64_t)(c + 1) * nblk] : total_rows;
    cls[2 * c] = start;
    cls[2 * c + 1] = end - start;
  }
}

__device__ __forceinline__ int wave_sum_i(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// SELF_SCAN: `offs` holds the raw class-major counts; every block sums the counts of all
// blocks (class totals) and of the blocks before it, and block 0 writes cls.  Otherwise
// `offs` is the scanned histogram and cls was written by the scan.
template <bool SELF_SCAN>
__global__ __launch_bounds__(kBucketThreads) void k_class_place(int64_t m, const int64_t *__restrict__ ptr,
                                                                const uint8_t *__restrict__ mask, int k,
                                                                int64_t split_min, const int32_t *__restrict__ offs,
                                                                RowRef *__restrict__ list, int64_t *__restrict__ cls) {
  __shared__ int wcnt[kBucketThreads / kWave][kNumClasses];
  __shared__ int run[kNumClasses];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the wave's rows first: their loads are in flight while the block derives its offsets
  const int64_t wbase = (int64_t)blockIdx.x * kRowsPerBlock + (int64_t)w * kRowsPerWave;
  WaveRows r;
  wave_rows_issue(r, m, ptr, mask, wbase, lane);
  if constexpr (SELF_SCAN) {
    __shared__ int tot[kNumClasses], pre[kNumClasses];
    const int nblk = (int)gridDim.x, me = (int)blockIdx.x;
    // wave w sums classes w, w + 8, w + 16: every count it needs is loaded before any is added
    // (one round trip to L2 instead of one per class and per 64 blocks)
    constexpr int WV = kBucketThreads / kWave, CW = (kNumClasses + WV - 1) / WV, BL = kSelfScanMaxBlocks / kWave;
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(offs, (uint64_t)kNumClasses * nblk * sizeof(int32_t));
    int h[CW][BL];
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w + WV * j < kNumClasses ? w + WV * j : kNumClasses - 1;
#pragma unroll
      for (int i = 0; i < BL; ++i) h[j][i] = bload_i32(ro, (c * nblk + lane + kWave * i) * (int)sizeof(int32_t));
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w + WV * j;
      int t = 0, p = 0;
#pragma unroll
      for (int i = 0; i < BL; ++i) {
        const int b = lane + kWave * i;
        const int x = b < nblk ? h[j][i] : 0;
        t += x;
        p += b < me ? x : 0;
      }
      t = wave_sum_i(t);
      p = wave_sum_i(p);
      if (lane == 0 && c < kNumClasses) {
        tot[c] = t;
        pre[c] = p;
      }
    }
    __syncthreads();
    if (tid < kNumClasses) {
      int start = 0;
      for (int c = 0; c < tid; ++c) start += tot[c];
      run[tid] = start + pre[tid];
      if (me == 0) {
        cls[2 * tid] = start;
        cls[2 * tid + 1] = tot[tid];
      }
    }
  } else {
    if (tid < kNumClasses) run[tid] = offs[(int64_t)tid * gridDim.x + blockIdx.x];
  }
  // Each wave places its own contiguous rows: first its per-class counts (lane cc holds class
  // cc), then, from its start within the block's run, the rows in order with ballot ranks.
  wave_rows_classify(r, k, split_min);
  const unsigned present = wave_classes_present(r);
  const int mine = wave_class_counts(r, lane, present);
  if (lane < kNumClasses) wcnt[w][lane] = mine;
  __syncthreads();
  int pos = 0;
  if (lane < kNumClasses) {
    pos = run[lane];
    for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][lane];
  }
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int c = r.c[p];
    int rank = 0, add = 0;
    for (unsigned b = present; b; b &= b - 1) {
      const int cc = __builtin_ctz(b);
      const unsigned long long bm = __ballot(c == cc);
      if (c == cc) rank = __popcll(bm & below);
      if (lane == cc) add = __popcll(bm);
    }
    const int base = __shfl(pos, c < 0 ? 0 : c, kWave);
    if (c >= 0) list[base + rank] = RowRef{(int32_t)(wbase + p * kWave + lane), r.cnt[p], r.beg[p]};
    pos += add;
  }
}
open_status bucket_rows_into(open_ctx *ctx, int64_t m, const int64_t *row_ptr, int k, int32_t *hist, RowRef *list,
                             int64_t *cls, int64_t split_min, const uint8_t *mask) {
  const int nblk = (int)((m + kRowsPerBlock - 1) / kRowsPerBlock);
  if (m > 0) {
    OPEN_LAUNCH(ctx, "bucket_count", k_class_count, dim3(nblk), dim3(kBucketThreads), 0, m, row_ptr, mask, k,
                split_min, hist);
  }
  if (m > 0 && nblk <= kSelfScanMaxBlocks) {
    OPEN_LAUNCH(ctx, "bucket_place", k_class_place<true>, dim3(nblk), dim3(kBucketThreads), 0, m, row_ptr, mask,
                k, split_min, (const int32_t *)hist, list, cls);
  } else {
    OPEN_LAUNCH(ctx, "bucket_scan", k_class_scan, dim3(1), dim3(1024), 0, hist, nblk, cls);
    if (m > 0) {
      OPEN_LAUNCH(ctx, "bucket_place", k_class_place<false>, dim3(nblk), dim3(kBucketThreads), 0, m, row_ptr, mask,
                  k, split_min, (const int32_t *)hist, list, cls);
    }
  }
  return OPEN_OK;
}

int64_t bucket_hist_ints(int64_t m) {
  const int64_t nblk = (m + kRowsPerBlock - 1) / kRowsPerBlock;
  return (int64_t)kNumClasses * (nblk > 0 ? nblk : 1);
}

open_status bucket_rows(open_ctx *ctx, int64_t m, const int64_t *row_ptr, int k, RowRef **list, int64_t **cls,
                        int64_t split_min, const uint8_t *mask) {
  void *hist = nullptr, *lst = nullptr, *c = nullptr;
  open_status st;
  if ((st = ws_get(ctx, open_ctx::WS_HIST, sizeof(int32_t) * (size_t)bucket_hist_ints(m), &hist))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_LIST, sizeof(RowRef) * (size_t)(m > 0 ? m : 1), &lst))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_CLS, sizeof(int64_t) * 2 * kNumClasses, &c))) return st;
  if ((st = bucket_rows_into(ctx, m, row_ptr, k, (int32_t *)hist, (RowRef *)lst, (int64_t *)c, split_min, mask)))
    return st;
  *list = (RowRef *)lst;
  *cls = (int64_t *)c;
  return OPEN_OK;
}

}  // namespace openk
