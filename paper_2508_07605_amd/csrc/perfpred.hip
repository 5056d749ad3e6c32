// Offline performance predictor (Section III-A.2, "Performance Prediction Model"), batched over
// profiled runs: each run's seven features (CPU cap, GPU cap, memory throughput, IPS, SM clock,
// DRAM active, FP active) map to the run's normalized performance,
//
//   z = (x - mu) * rs,  h1 = ReLU(W1 z + b1),  h2 = ReLU(W2 h1 + b2),  y = w3 . h2 + b3,
//
// with two hidden layers of 64 units.  W1 (64 x 7) and W2 (64 x 64) are used in bfloat16
// (round to nearest even); everything else is float32.  A run with a non-finite feature gets
// y = NaN.
//
// One wavefront per tile of 32 runs, on BF16 MFMA v_mfma_f32_32x32x16_bf16 with the runs along
// the 32 output columns and the hidden units along the rows.  The activations are not rounded
// to bfloat16: each is split into a bfloat16 part and a bfloat16 remainder (a = hi + lo up to
// 2^-18 |a|) and both are multiplied, so the only rounding beyond float32 is the weights'.
//   layer 1: k = 8 g + t pairs weight column t with the feature parts of half g (g = 0 the
//            bfloat16 parts, g = 1 the remainders); bias b1 enters as the accumulator.
//   layer 2: the hidden index of slot (g, t) in step s = 2 bk + p is chosen as the row that
//            the layer-1 result already holds in that lane, 32 bk + 8 (2p + t/4) + 4 g + t%4,
//            so h1 feeds the next MFMA without moving between lanes; W2 is permuted to match.
//   layer 3: a per-lane dot product over the 32 held units, then the two halves are added.
#include "common.h"

namespace openk {

typedef __bf16 pbf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));

constexpr int kPF = 7;   // features
constexpr int kPH = 64;  // hidden units per layer

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const pbf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
// a = hi + lo (bfloat16 parts, packed in pairs); the remainder is exact in float32
__device__ __forceinline__ void split_pair(float a, float b, uint32_t &hi, uint32_t &lo) {
  hi = pack_bf16(a, b);
  const float ha = __builtin_bit_cast(float, hi << 16), hb = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = pack_bf16(a - ha, b - hb);
}
__device__ __forceinline__ f16 mfma_bf16(uint4 a, uint4 b, f16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pbf16x8, a), __builtin_bit_cast(pbf16x8, b), c,
                                                 0, 0, 0);
}

__global__ __launch_bounds__(256) void k_perf_predict(int64_t n, const float *__restrict__ X,
                                                      const float *__restrict__ mu, const float *__restrict__ rs,
                                                      const float *__restrict__ W1, const float *__restrict__ b1,
                                                      const float *__restrict__ W2, const float *__restrict__ b2,
                                                      const float *__restrict__ w3, const float *__restrict__ b3,
                                                      float *__restrict__ y) {
  const int lane = threadIdx.x & 63, i32 = lane & 31, g = lane >> 5;
  // rows of the 32 x 32 result held by this lane: 8 (v/4) + 4 g + v%4
  auto rr = [&](int v) { return 8 * (v >> 2) + 4 * g + (v & 3); };
  // layer-1 weights, A operand of row block bk: W1[32 bk + i32][t] for t < 7, 0 for t = 7
  uint4 a1[2];
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) {
    const float *w = W1 + (32 * bk + i32) * kPF;
    a1[bk] = uint4{pack_bf16(w[0], w[1]), pack_bf16(w[2], w[3]), pack_bf16(w[4], w[5]), pack_bf16(w[6], 0.f)};
  }
  // layer-2 weights, A operand of output block ob and step s = 2 bk + p: slot t of half g is
  // input unit 32 bk + 8 (2p + t/4) + 4 g + t%4
  uint4 a2[2][4];
#pragma unroll
  for (int ob = 0; ob < 2; ++ob)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float *w = W2 + (32 * ob + i32) * kPH + 32 * (s >> 1) + 4 * g;
      const int p = s & 1;
      uint32_t q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t0 = 2 * u, t1 = 2 * u + 1;
        q[u] = pack_bf16(w[8 * (2 * p + t0 / 4) + t0 % 4], w[8 * (2 * p + t1 / 4) + t1 % 4]);
      }
      a2[ob][s] = uint4{q[0], q[1], q[2], q[3]};
    }
  f16 c1[2], c2[2], w3r[2];
#pragma unroll
  for (int bk = 0; bk < 2; ++bk)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      c1[bk][v] = b1[32 * bk + rr(v)];
      c2[bk][v] = b2[32 * bk + rr(v)];
      w3r[bk][v] = w3[32 * bk + rr(v)];
    }
  float muf[kPF], rsf[kPF];
#pragma unroll
  for (int f = 0; f < kPF; ++f) {
    muf[f] = mu[f];
    rsf[f] = rs[f];
  }
  const float bias3 = b3[0];

  const int64_t ntiles = (n + 31) >> 5;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t tile0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  // the features of the next tile are loaded while the current one is computed
  float xn[kPF];
#pragma unroll
  for (int f = 0; f < kPF; ++f) xn[f] = (tile0 << 5) + i32 < n ? X[((tile0 << 5) + i32) * kPF + f] : 0.f;
  for (int64_t tile = tile0; tile < ntiles; tile += nw) {
    const int64_t e = (tile << 5) + i32, en = ((tile + nw) << 5) + i32;
    float z[8];
    bool finite = true;
#pragma unroll
    for (int f = 0; f < kPF; ++f) {
      const float x = xn[f];
      xn[f] = en < n ? X[en * kPF + f] : 0.f;
      finite = finite && __builtin_isfinite(x);
      z[f] = (x - muf[f]) * rsf[f];
    }
    z[7] = 0.f;
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) split_pair(z[2 * u], z[2 * u + 1], hi[u], lo[u]);
    const uint4 bx = g == 0 ? uint4{hi[0], hi[1], hi[2], hi[3]} : uint4{lo[0], lo[1], lo[2], lo[3]};
    f16 d1[2];
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) d1[bk] = mfma_bf16(a1[bk], bx, c1[bk]);
    f16 d2[2] = {c2[0], c2[1]};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int bk = s >> 1, p = s & 1;
      uint32_t hh[4], hl[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float x0 = __builtin_fmaxf(d1[bk][8 * p + 2 * u], 0.f);
        const float x1 = __builtin_fmaxf(d1[bk][8 * p + 2 * u + 1], 0.f);
        split_pair(x0, x1, hh[u], hl[u]);
      }
      const uint4 bh = uint4{hh[0], hh[1], hh[2], hh[3]}, bl = uint4{hl[0], hl[1], hl[2], hl[3]};
#pragma unroll
      for (int ob = 0; ob < 2; ++ob) {
        d2[ob] = mfma_bf16(a2[ob][s], bh, d2[ob]);
        d2[ob] = mfma_bf16(a2[ob][s], bl, d2[ob]);
      }
    }
    float acc = 0.f;
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc = __builtin_fmaf(w3r[ob][v], __builtin_fmaxf(d2[ob][v], 0.f), acc);
    acc += __shfl_xor(acc, 32, kWave);
    if (g == 0 && e < n) y[e] = finite ? acc + bias3 : __builtin_nanf("");
  }
}

}  // namespace openk

using namespace openk;

extern "C" open_status open_perf_predict(open_ctx *ctx, const float *X, int64_t n_runs, const float *mu,
                                         const float *rs, const float *W1, const float *b1, const float *W2,
                                         const float *b2, const float *w3, const float *b3, float *y) {
  if (!ctx) return OPEN_E_INVALID;
  if (n_runs < 0) return fail(ctx, OPEN_E_INVALID, "negative run count");
  if (n_runs == 0) return OPEN_OK;
  if (!X || !mu || !rs || !W1 || !b1 || !W2 || !b2 || !w3 || !b3 || !y)
    return fail(ctx, OPEN_E_INVALID, "null pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int64_t tiles = (n_runs + 31) / 32;
  const int64_t cap = (int64_t)ctx->num_cu * 8;  // waves
  const int64_t waves = tiles < cap ? tiles : cap;
  OPEN_LAUNCH(ctx, "perf_predict", k_perf_predict, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, n_runs, X, mu,
              rs, W1, b1, W2, b2, w3, b3, y);
  return OPEN_OK;
}
