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
//            bfloat16 parts, g = 1 the remainders); the bias b1 rides in slot t = 7 against
//            a constant feature of 1, again as a bfloat16 part and its remainder.
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
// max(x, 0) on the bit pattern: negative floats are negative integers (one integer max, no
// NaN canonicalisation)
__device__ __forceinline__ float relu(float x) {
  const int i = __builtin_bit_cast(int, x);
  return __builtin_bit_cast(float, i > 0 ? i : 0);
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
  // the 32 x 32 results hold rows 8 (v/4) + 4 g + v%4 of the tile in register v of the lane
  // layer-1 weights, A operand of row block bk: W1[32 bk + i32][t] for t < 7; slot t = 7 holds
  // the bias, its bfloat16 part in half 0 and the remainder in half 1 (times a feature of 1)
  uint4 a1[2];
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) {
    const float *w = W1 + (32 * bk + i32) * kPF;
    uint32_t bh, bl;
    split_pair(b1[32 * bk + i32], 0.f, bh, bl);
    a1[bk] = uint4{pack_bf16(w[0], w[1]), pack_bf16(w[2], w[3]), pack_bf16(w[4], w[5]),
                   pack_bf16(w[6], __builtin_bit_cast(float, (g == 0 ? bh : bl) << 16))};
  }
  // layer-2 weights, A operand of output block ob and step s = 2 bk + p: slot t of half g is
  // input unit 32 bk + 8 (2p + t/4) + 4 g + t%4.  Each lane's operands depend on the lane
  // only, so the block keeps one copy in LDS: la2[ob][s][lane].
  __shared__ uint4 la2[2][4][kWave];
  for (int q = threadIdx.x; q < 2 * 4 * kWave; q += blockDim.x) {
    const int ob = q / (4 * kWave), s = (q / kWave) % 4, l = q % kWave, li = l & 31, lg = l >> 5;
    const float *w = W2 + (32 * ob + li) * kPH + 32 * (s >> 1) + 4 * lg;
    const int p = s & 1;
    uint32_t qq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t0 = 2 * u, t1 = 2 * u + 1;
      qq[u] = pack_bf16(w[8 * (2 * p + t0 / 4) + t0 % 4], w[8 * (2 * p + t1 / 4) + t1 % 4]);
    }
    la2[ob][s][l] = uint4{qq[0], qq[1], qq[2], qq[3]};
  }
  // b2 and w3 stay in LDS (read per tile, four consecutive rows at a time), which keeps the
  // register count low enough for more wavefronts per SIMD
  __shared__ f4 lb2[16], lw3[16];
  if (threadIdx.x < 64) {
    reinterpret_cast<float *>(lb2)[threadIdx.x] = b2[threadIdx.x];
  } else if (threadIdx.x < 128) {
    reinterpret_cast<float *>(lw3)[threadIdx.x - 64] = w3[threadIdx.x - 64];
  }
  __syncthreads();
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
    z[7] = 1.f;  // multiplies the layer-1 bias parts
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) split_pair(z[2 * u], z[2 * u + 1], hi[u], lo[u]);
    lo[3] = (lo[3] & 0xffffu) | 0x3f800000u;  // slot 7 is 1 in both halves
    const uint4 bx = g == 0 ? uint4{hi[0], hi[1], hi[2], hi[3]} : uint4{lo[0], lo[1], lo[2], lo[3]};
    f16 d1[2];
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) d1[bk] = mfma_bf16(a1[bk], bx, f16{});
    f16 d2[2];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
      for (int a = 0; a < 4; ++a) {  // rows 32 ob + 8 a + 4 g + 0..3
        const f4 b = lb2[8 * ob + 2 * a + g];
        d2[ob][4 * a] = b[0];
        d2[ob][4 * a + 1] = b[1];
        d2[ob][4 * a + 2] = b[2];
        d2[ob][4 * a + 3] = b[3];
      }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int bk = s >> 1, p = s & 1;
      uint32_t hh[4], hl[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float x0 = relu(d1[bk][8 * p + 2 * u]);
        const float x1 = relu(d1[bk][8 * p + 2 * u + 1]);
        split_pair(x0, x1, hh[u], hl[u]);
      }
      const uint4 bh = uint4{hh[0], hh[1], hh[2], hh[3]}, bl = uint4{hl[0], hl[1], hl[2], hl[3]};
#pragma unroll
      for (int ob = 0; ob < 2; ++ob) {
        const uint4 w = la2[ob][s][lane];
        d2[ob] = mfma_bf16(w, bh, d2[ob]);
        d2[ob] = mfma_bf16(w, bl, d2[ob]);
      }
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const f4 w = lw3[8 * ob + 2 * a + g];
#pragma unroll
        for (int c = 0; c < 4; ++c) part[c] = __builtin_fmaf(w[c], relu(d2[ob][4 * a + c]), part[c]);
      }
    float acc = (part[0] + part[1]) + (part[2] + part[3]);
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
  const int64_t cap = (int64_t)ctx->num_cu * 16;  // waves
  const int64_t waves = tiles < cap ? tiles : cap;
  OPEN_LAUNCH(ctx, "perf_predict", k_perf_predict, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, n_runs, X, mu,
              rs, W1, b1, W2, b2, w3, b3, y);
  return OPEN_OK;
}
