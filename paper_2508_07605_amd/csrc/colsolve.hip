// Split-K ridge solve of long rows (weighted-lambda ALS, the completion step of Section III-B):
//   x_i = (sum_{j in O_i} f_j f_j^T + lambda w_i I)^-1  sum_{j in O_i} r_ij f_j
// for the rows with at least kSplitMin observations (size class kSplitClass of the
// bucketing).  These are the columns of the ALS column half-sweep (solved on the column
// view, F = U): a few hundred of them hold most of the observed entries, so one system per
// lane group would leave the chip idle; instead
//   1. k_split_prefix  numbers the chunks of kSplitChunk observations of every long column;
//   2. k_split_gram    one wavefront per chunk forms the partial Gram matrix on FP32 MFMA
//                      (the observation index is the contraction index, so one register of
//                      u values is both operands) and the partial right-hand side;
//   3. k_split_solve   one wavefront per column sums its partials in chunk order (the result
//                      does not depend on scheduling), adds the ridge and solves by LDL^T in LDS.
#include "common.h"

namespace openk {

typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int kSplitChunk = 1024;
constexpr int kXcds = 8;  // accelerator complex dies of the MI355X, each with its own L2
constexpr int kPrefixThreads = 1024;

// MFMA geometry per rank: tile TK (16: v_mfma_f32_16x16x4f32, 32: v_mfma_f32_32x32x2f32),
// observations per instruction OBS, 32x32 blocks NB (rank 64 keeps the three lower blocks)
template <int K>
struct SplitGeo {
  static constexpr int TK = K <= 16 ? 16 : 32;
  static constexpr int OBS = 64 / TK;
  static constexpr int NB = K == 64 ? 3 : 1;
  static constexpr int GRAM = NB * TK * TK;          // partial Gram floats (MFMA register order)
  static constexpr int RHS = K == 64 ? 128 : 64;      // partial rhs floats (one per lane and half)
  static constexpr int PST = GRAM + RHS;              // floats per chunk
};

int split_part_floats(int k) {
  switch (k) {
    case 8: return SplitGeo<8>::PST;
    case 16: return SplitGeo<16>::PST;
    case 32: return SplitGeo<32>::PST;
    default: return SplitGeo<64>::PST;
  }
}

// chunk_start[i] = first chunk of long column i (list position cls[2 kSplitClass] + i),
// chunk_start[count] = total chunks
__global__ __launch_bounds__(kPrefixThreads) void k_split_prefix(const RowRef *__restrict__ list,
                                                                 const int64_t *__restrict__ cls,
                                                                 int64_t *__restrict__ chunk_start) {
  __shared__ int64_t part[kPrefixThreads];
  const int64_t s0 = cls[2 * kSplitClass], cnt = cls[2 * kSplitClass + 1];
  const int64_t per = (cnt + kPrefixThreads - 1) / kPrefixThreads;
  const int64_t b0 = threadIdx.x * per, b1 = b0 + per < cnt ? b0 + per : cnt;
  int64_t s = 0;
  for (int64_t i = b0; i < b1; ++i) s += (list[s0 + i].cnt + kSplitChunk - 1) / kSplitChunk;
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kPrefixThreads; off <<= 1) {
    const int64_t x = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int64_t i = b0; i < b1; ++i) {
    chunk_start[i] = run;
    run += (list[s0 + i].cnt + kSplitChunk - 1) / kSplitChunk;
  }
  if (threadIdx.x == kPrefixThreads - 1) chunk_start[cnt] = part[kPrefixThreads - 1];
  // largest chunk count of a row, for the chunk-major visiting order of k_split_gram
  __shared__ int64_t mx[kPrefixThreads];
  int64_t m1 = 0;
  for (int64_t i = b0; i < b1; ++i) {
    const int64_t c = (list[s0 + i].cnt + kSplitChunk - 1) / kSplitChunk;
    m1 = c > m1 ? c : m1;
  }
  mx[threadIdx.x] = m1;
  __syncthreads();
  for (int off = kPrefixThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off && mx[threadIdx.x + off] > mx[threadIdx.x]) mx[threadIdx.x] = mx[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) chunk_start[cnt + 1] = mx[0];
}

// Partial Gram and rhs of chunks g = wave, wave + waves, ... (persistent).  Lane l supplies
// dimension l % TK of observation l / TK of each MFMA step.
template <int K>
__global__ __launch_bounds__(256) void k_split_gram(const float *__restrict__ Uf, const int32_t *__restrict__ ri,
                                                    const float *__restrict__ cv, const RowRef *__restrict__ list,
                                                    const int64_t *__restrict__ cls,
                                                    const int64_t *__restrict__ chunk_start, int nF,
                                                    float *__restrict__ part, int32_t *__restrict__ cflag) {
  using G = SplitGeo<K>;
  constexpr int TK = G::TK, OBS = G::OBS, UNR = 16;
  // per wavefront: the chunk's indices and values, staged once with coalesced loads
  __shared__ int jl_all[4][kSplitChunk];
  __shared__ float rl_all[4][kSplitChunk];
  int *jl = jl_all[threadIdx.x >> 6];
  float *rl = rl_all[threadIdx.x >> 6];
  const int64_t s0 = cls[2 * kSplitClass], cnt = cls[2 * kSplitClass + 1];
  if (cnt == 0) return;
  const int64_t cmax = chunk_start[cnt + 1];
  const __amdgpu_buffer_rsrc_t urs = make_rsrc(Uf, (uint64_t)nF * K * sizeof(float));
  const int lane = threadIdx.x & 63;
  const int d = lane % TK, o = lane / TK;  // dimension and observation slot of this lane
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  // Visiting order.  Virtual index v = c * cnt + row runs chunk position-major, so wavefronts
  // running together take the same chunk position of many rows, whose gathered factor rows
  // then come from a narrow index range (the column view keeps entries sorted by row).
  // Workgroups are dealt to the 8 XCDs round-robin: each XCD walks its own slabs of
  // consecutive v, so the range it gathers from stays within its L2.
  const int64_t total_v = cmax * cnt;
  const bool xcd_order = gridDim.x % kXcds == 0;
  const int64_t slab = xcd_order ? (int64_t)(gridDim.x / kXcds) * (blockDim.x >> 6) : nw;
  const int64_t wx = xcd_order ? (int64_t)(blockIdx.x / kXcds) * (blockDim.x >> 6) + (threadIdx.x >> 6)
                               : (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t first = xcd_order ? blockIdx.x % kXcds : 0, stride = xcd_order ? kXcds : 1;
  for (int64_t sl = first; sl * slab < total_v; sl += stride) {
    const int64_t v = sl * slab + wx;
    if (v >= total_v) continue;
    const int64_t lo = v % cnt, c = v / cnt;
    const int64_t nch = chunk_start[lo + 1] - chunk_start[lo];
    if (c >= nch) continue;  // this row has fewer chunks (wave-uniform)
    const int64_t g = chunk_start[lo] + c;
    const RowRef rr = list[s0 + lo];
    const int64_t c0 = c * kSplitChunk;
    const int64_t beg = rr.beg + c0;
    const int len = (int)((int64_t)rr.cnt - c0 < kSplitChunk ? (int64_t)rr.cnt - c0 : kSplitChunk);
    // two accumulator sets (even and odd MFMA steps) so consecutive MFMAs do not depend on
    // each other; summed once at the end
    f16v acc[G::NB], acc2[G::NB];
    float bl = 0.f, bh = 0.f;
    for (int b = 0; b < G::NB; ++b) acc[b] = acc2[b] = f16v{};
    f4 acc16 = {0.f, 0.f, 0.f, 0.f}, acc16b = {0.f, 0.f, 0.f, 0.f};
    int flags = 0;  // 1: non-finite value, 2: index outside [0, nF)
    // software pipeline: the operands of batch t + 1 load while batch t feeds the MFMAs
    // stage: entry t of the chunk -> (jl[t], rl[t]); rejected or absent entries get j = -1
    __builtin_amdgcn_wave_barrier();  // the previous chunk's reads are done
#pragma unroll
    for (int i = 0; i < kSplitChunk / 64; ++i) {
      const int t = i * 64 + lane;
      const bool in = t < len;
      const int j = in ? ri[beg + t] : -1;
      const float r = in ? cv[beg + t] : 0.f;
      const bool jok = j >= 0 && j < nF;
      if (in && !jok) flags |= 2;
      if (in && !__builtin_isfinite(r)) flags |= 1;
      jl[t] = jok ? j : -1;
      rl[t] = r;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float ul[UNR], uh[UNR], rv[UNR];
    // factor rows through a bounds-checked buffer resource: the row index -1 of absent or
    // rejected entries reads zeros, so no per-element tests remain
    auto load = [&](int t0) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int t = t0 + u * OBS + o;  // < kSplitChunk; entries past len were staged as -1
        const int j = jl[t];
        rv[u] = rl[t];
        const uint32_t off = (uint32_t)(j * K + d) * 4u;
        ul[u] = (K >= TK || d < K) ? bload_f32(urs, d < K ? off : 0xffffffffu) : 0.f;
        if constexpr (K == 64)
          uh[u] = bload_f32(urs, off + 128u);
        else
          uh[u] = 0.f;
      }
    };
    load(0);
    for (int t0 = 0; t0 < len; t0 += OBS * UNR) {
      float cl[UNR], ch[UNR], cr[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        cl[u] = ul[u];
        ch[u] = uh[u];
        cr[u] = rv[u];
      }
      if (t0 + OBS * UNR < len) load(t0 + OBS * UNR);
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        f16v *A = (u & 1) ? acc2 : acc;
        if constexpr (TK == 16) {
          if (u & 1)
            acc16b = __builtin_amdgcn_mfma_f32_16x16x4f32(cl[u], cl[u], acc16b, 0, 0, 0);
          else
            acc16 = __builtin_amdgcn_mfma_f32_16x16x4f32(cl[u], cl[u], acc16, 0, 0, 0);
        } else {
          A[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(cl[u], cl[u], A[0], 0, 0, 0);
          if constexpr (K == 64) {
            A[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ch[u], cl[u], A[1], 0, 0, 0);  // rows 32.., cols ..31
            A[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(ch[u], ch[u], A[2], 0, 0, 0);
          }
        }
        bl = __builtin_fmaf(cr[u], cl[u], bl);
        if constexpr (K == 64) bh = __builtin_fmaf(cr[u], ch[u], bh);
      }
    }
    for (int b = 0; b < G::NB; ++b) acc[b] += acc2[b];
    acc16 += acc16b;
    float *dst = part + g * G::PST;
    if constexpr (TK == 16) {
      for (int v = 0; v < 4; ++v) dst[v * 64 + lane] = acc16[v];
    } else {
      for (int b = 0; b < G::NB; ++b)
        for (int v = 0; v < 16; ++v) dst[(b * 16 + v) * 64 + lane] = acc[b][v];
    }
    dst[G::GRAM + lane] = bl;
    if constexpr (K == 64) dst[G::GRAM + 64 + lane] = bh;
    // wave OR of the flags
    const unsigned long long f1 = __ballot(flags & 1), f2 = __ballot(flags & 2);
    if (lane == 0) cflag[g] = (f1 ? 1 : 0) | (f2 ? 2 : 0);
  }
}

// One wavefront per long column: reduce its partials, add the ridge, LDL^T in LDS, solve.
template <int K>
__global__ __launch_bounds__(64) void k_split_solve(const RowRef *__restrict__ list, const int64_t *__restrict__ cls,
                                                    const int64_t *__restrict__ chunk_start,
                                                    const float *__restrict__ part,
                                                    const int32_t *__restrict__ cflag, float lambda, int weighted,
                                                    float *__restrict__ X, int32_t *__restrict__ status) {
  using G = SplitGeo<K>;
  constexpr int TK = G::TK, LDA = K + 1;
  __shared__ float A[K * LDA];
  __shared__ float b[K];
  __shared__ int bad;
  const int64_t s0 = cls[2 * kSplitClass], cnt = cls[2 * kSplitClass + 1];
  const int64_t i = blockIdx.x;
  if (i >= cnt) return;
  const RowRef rr = list[s0 + i];
  const int lane = threadIdx.x;
  const int64_t g0 = chunk_start[i], g1 = chunk_start[i + 1];
  // sum of the partials in chunk order, in the MFMA register layout
  float gs[G::NB * (TK == 16 ? 4 : 16)];
  float bsum[K == 64 ? 2 : 1];
  for (int e = 0; e < G::NB * (TK == 16 ? 4 : 16); ++e) gs[e] = 0.f;
  bsum[0] = 0.f;
  if constexpr (K == 64) bsum[1] = 0.f;
  int flags = 0;
  for (int64_t g = g0; g < g1; ++g) {
    flags |= cflag[g];
    const float *src = part + g * G::PST;
    for (int e = 0; e < G::NB * (TK == 16 ? 4 : 16); ++e) gs[e] += src[e * 64 + lane];
    bsum[0] += src[G::GRAM + lane];
    if constexpr (K == 64) bsum[1] += src[G::GRAM + 64 + lane];
  }
  // scatter to the dense lower triangle (and the diagonal blocks' upper parts, unused)
  if constexpr (TK == 16) {
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * (lane / 16) + v, c = lane % 16;
      if (r < K && c < K) A[r * LDA + c] = gs[v];
    }
  } else {
    for (int blk = 0; blk < G::NB; ++blk) {
      const int ro = blk >= 1 ? 32 : 0, co = blk == 2 ? 32 : 0;
      for (int v = 0; v < 16; ++v) {
        const int r = ro + 8 * (v / 4) + 4 * (lane / 32) + (v % 4), c = co + lane % 32;
        A[r * LDA + c] = gs[blk * 16 + v];
      }
    }
  }
  // rhs: lane l holds dimension l % TK of observation slot l / TK
  {
    __shared__ float bp[K == 64 ? 128 : 64];
    bp[lane] = bsum[0];
    if constexpr (K == 64) bp[64 + lane] = bsum[1];
    __syncthreads();
    if (lane < K) {
      float s = 0.f;
      if constexpr (K == 64) {
        const int dd = lane % 32, half = lane / 32;
        s = bp[half * 64 + dd] + bp[half * 64 + 32 + dd];
      } else {
        for (int q = 0; q < 64 / TK; ++q) s += bp[q * TK + lane];
      }
      b[lane] = s;
    }
  }
  if (lane == 0) bad = 0;
  __syncthreads();
  const float reg = lambda * (weighted ? (float)rr.cnt : 1.0f);
  if (lane < K) A[lane * LDA + lane] += reg;
  __syncthreads();
  // LDL^T, right-looking; lane r updates row r of the lower triangle
  for (int p = 0; p < K; ++p) {
    const float dp = A[p * LDA + p];
    if (lane == 0 && !(dp > 0.f && __builtin_isfinite(dp))) bad = 1;
    const float inv = 1.0f / dp;
    float l = 0.f;
    if (lane > p && lane < K) l = A[lane * LDA + p] * inv;
    __syncthreads();
    if (lane > p && lane < K) {
      for (int c = p + 1; c <= lane; ++c) A[lane * LDA + c] -= l * A[c * LDA + p];
    }
    __syncthreads();
    if (lane > p && lane < K) A[lane * LDA + p] = l;
    __syncthreads();
  }
  // forward (unit L), diagonal, backward (L^T)
  for (int p = 0; p < K; ++p) {
    const float bpv = b[p];
    __syncthreads();
    if (lane > p && lane < K) b[lane] -= A[lane * LDA + p] * bpv;
    __syncthreads();
  }
  if (lane < K) b[lane] /= A[lane * LDA + lane];
  __syncthreads();
  for (int p = K - 1; p >= 0; --p) {
    const float xp = b[p];
    __syncthreads();
    if (lane < p) b[lane] -= A[p * LDA + lane] * xp;
    __syncthreads();
  }
  const bool good = !bad && flags == 0;
  if (lane < K) X[(int64_t)rr.row * K + lane] = good ? b[lane] : 0.f;
  if (status && lane == 0)
    status[rr.row] = (flags & 2) ? OPEN_ROW_BADINDEX
                     : (flags & 1) ? OPEN_ROW_NONFINITE
                     : bad        ? OPEN_ROW_NONPOS_PIVOT
                                  : OPEN_ROW_OK;
}

template <int K>
static open_status split_launch_k(open_ctx *ctx, const float *F, int nF, const int32_t *ri, const float *cv,
                                  const RowRef *list, const int64_t *cls, int64_t *chunk_start, float *part,
                                  int32_t *cflag, float lambda, int weighted, float *X, int32_t *status,
                                  int64_t max_rows) {
  OPEN_LAUNCH(ctx, "split_prefix", k_split_prefix, dim3(1), dim3(kPrefixThreads), 0, list, cls, chunk_start);
  OPEN_LAUNCH(ctx, "split_gram", k_split_gram<K>, dim3(ctx->num_cu * 4), dim3(256), 0, F, ri, cv, list, cls,
              chunk_start, nF, part, cflag);
  OPEN_LAUNCH(ctx, "split_solve", k_split_solve<K>, dim3((unsigned)max_rows), dim3(64), 0, list, cls, chunk_start,
              part, cflag, lambda, weighted, X, status);
  return OPEN_OK;
}

open_status splitk_launch(open_ctx *ctx, const float *F, int nF, int k, const int32_t *idx, const float *val,
                          float lambda, int weighted, const RowRef *list, const int64_t *cls, float *X,
                          int32_t *status, int64_t m, int64_t nnz) {
  // at most nnz / kSplitMin long rows, each with at most len / kSplitChunk + 1 chunks
  int64_t max_rows = nnz / kSplitMin + 1;
  if (max_rows > m) max_rows = m;
  if (max_rows < 1) return OPEN_OK;
  if (max_rows > INT32_MAX) return fail(ctx, OPEN_E_UNSUPPORTED, "too many long rows");
  const int64_t max_chunks = nnz / kSplitChunk + max_rows + 1;
  void *cs = nullptr, *pt = nullptr, *cf = nullptr;
  open_status st;
  // chunk_start: one entry per long row, the total, and the largest chunk count
  if ((st = ws_get(ctx, open_ctx::WS_SPLIT_START, sizeof(int64_t) * (size_t)(max_rows + 2), &cs))) return st;
  if ((st = ws_get(ctx, open_ctx::WS_SPLIT_PART, sizeof(float) * (size_t)max_chunks * split_part_floats(k), &pt)))
    return st;
  if ((st = ws_get(ctx, open_ctx::WS_SPLIT_FLAG, sizeof(int32_t) * (size_t)max_chunks, &cf))) return st;
  int64_t *c = (int64_t *)cs;
  float *p = (float *)pt;
  int32_t *f = (int32_t *)cf;
  switch (k) {
    case 8: return split_launch_k<8>(ctx, F, nF, idx, val, list, cls, c, p, f, lambda, weighted, X, status, max_rows);
    case 16: return split_launch_k<16>(ctx, F, nF, idx, val, list, cls, c, p, f, lambda, weighted, X, status, max_rows);
    case 32: return split_launch_k<32>(ctx, F, nF, idx, val, list, cls, c, p, f, lambda, weighted, X, status, max_rows);
    case 64: return split_launch_k<64>(ctx, F, nF, idx, val, list, cls, c, p, f, lambda, weighted, X, status, max_rows);
    default: return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  }
}

}  // namespace openk
