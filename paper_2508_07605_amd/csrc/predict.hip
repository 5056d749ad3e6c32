// Fused prediction + energy-efficient cap selection (Algorithm 2, Section III-B.3).
//
// p_is = u_i . v_s is formed tile by tile on FP32 MFMA (v_mfma_f32_32x32x2_f32): a wavefront
// owns 32 rows, keeps their factor rows in registers (A operand) and streams the setting
// factors through LDS in blocks of 32 settings (B operand, stored transposed with a padded
// stride so the 32 lanes of a half-wave read distinct banks).  The epilogue applies the
// paper's rule to every element without materialising p:
//   p_base = p_ib                          (the same MFMA value the scan sees for s = b)
//   valid  = p > 0  and  1 - p / p_base <= gamma      (float32, correctly rounded division; as
//            the equivalent p >= t with t found once per row, the test being monotone in p)
//   E      = (c_s + g_s) / p: the least E is the greatest key p * iw_s, iw_s = 1 / (c_s + g_s)
//            (float32, one division per setting instead of one per element); the lowest s on
//            ties; the saving (E_base - E) / E_base with E = (c_s + g_s) / p of the pick
// Each lane scans its own settings in ascending order; the 32 lanes of a half-wave are then
// combined by (E, s) in a butterfly.  The full prediction P is written only when asked.
#include <math.h>

#include "common.h"

namespace openk {

typedef float f16v __attribute__((ext_vector_type(16)));

// V block s0 (32 settings x K) as K/8 floats per thread of a 256-thread block: load from global,
// then store transposed into LDS at stride LD (settings past n read as zero)
template <int K>
__device__ __forceinline__ void load_block(float (&t)[K / 8], const float *__restrict__ V, int n, int s0) {
#pragma unroll
  for (int i = 0; i < K / 8; ++i) {
    const int e = threadIdx.x + 256 * i, j = e / K, kk = e % K;
    t[i] = (s0 + j < n) ? V[(int64_t)(s0 + j) * K + kk] : 0.f;
  }
}
template <int K>
__device__ __forceinline__ void store_block(float *Vt, const float (&t)[K / 8]) {
  constexpr int LD = 33;
#pragma unroll
  for (int i = 0; i < K / 8; ++i) {
    const int e = threadIdx.x + 256 * i, j = e / K, kk = e % K;
    Vt[kk * LD + j] = t[i];
  }
}

template <int K>
__device__ __forceinline__ f16v tile(const float (&a)[K / 2], const float *Vt, int r, int h) {
  constexpr int H = K / 2, LD = 33;
  f16v acc = {};
#pragma unroll
  for (int s = 0; s < H; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], Vt[(h * H + s) * LD + r], acc, 0, 0, 0);
  return acc;
}

// The rule's validity test 1 - p / p_base <= gamma (float32, correctly rounded division and
// subtraction) is monotone in p for p_base > 0: fl(p / p_base) does not decrease as p grows and
// fl(1 - x) does not increase as x grows.  So it holds exactly for p >= t, t the least float
// for which it holds, found once per row from the real threshold (1 - gamma) p_base by stepping
// a few units in the last place (the two roundings move it by about two).
__device__ __forceinline__ bool loss_ok(float p, float pb, float gamma) { return (1.0f - p / pb) <= gamma; }
__device__ __forceinline__ float least_valid(float pb, float gamma) {
  float t = (1.0f - gamma) * pb;
  if (!(t > 0.f)) return __builtin_bit_cast(float, 1);  // gamma >= 1: every p > 0 passes
  auto step = [](float x, int d) { return __builtin_bit_cast(float, __builtin_bit_cast(int, x) + d); };
  for (int i = 0; i < 64 && loss_ok(step(t, -1), pb, gamma); ++i) t = step(t, -1);
  for (int i = 0; i < 64 && !loss_ok(t, pb, gamma); ++i) t = step(t, 1);
  return t;
}

template <int K>
__global__ __launch_bounds__(256) void k_predict_select(const float *__restrict__ U, int64_t m,
                                                        const float *__restrict__ V, int n,
                                                        const float *__restrict__ cap_c,
                                                        const float *__restrict__ cap_g, int base, float gamma,
                                                        float *__restrict__ P, int32_t *__restrict__ best_idx,
                                                        float *__restrict__ best_saving,
                                                        int32_t *__restrict__ status) {
  constexpr int H = K / 2, LD = 33;
  __shared__ float Vt[2][K * LD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + w) * 32;
  const int64_t grow = row0 + r;
  // A operand: lane (r, h) holds u_r[h*H .. h*H + H)
  float a[H];
#pragma unroll
  for (int s = 0; s < H; s += 4) {
    const f4 x = grow < m ? *reinterpret_cast<const f4 *>(U + grow * K + h * H + s) : f4{0.f, 0.f, 0.f, 0.f};
    a[s] = x[0];
    a[s + 1] = x[1];
    a[s + 2] = x[2];
    a[s + 3] = x[3];
  }
  // rows of this lane's 16 accumulators: 8*(v/4) + 4*h + v%4
  // baseline prediction from the same MFMA tile the scan uses
  const int sb0 = (base / 32) * 32, jb = base - sb0;
  float tb[K / 8];
  load_block<K>(tb, V, n, sb0);
  store_block<K>(Vt[1], tb);
  load_block<K>(tb, V, n, 0);  // the scan's first block
  __syncthreads();
  float pb[16], thr[16];
  {
    const f16v acc = tile<K>(a, Vt[1], r, h);
#pragma unroll
    for (int v = 0; v < 16; ++v) pb[v] = __shfl(acc[v], jb + 32 * h, 64);
  }
  // per row: valid(p) <=> p >= thr (thr > 0, so p > 0 follows; NaN when p_base <= 0: never)
#pragma unroll
  for (int v = 0; v < 16; ++v) thr[v] = pb[v] > 0.f ? least_valid(pb[v], gamma) : __builtin_nanf("");
  float bK[16], bP[16];  // the best key and its prediction
  int bS[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    bK[v] = -__builtin_inff();
    bP[v] = 0.f;
    bS[v] = -1;
  }
  store_block<K>(Vt[0], tb);
  if (32 < n) load_block<K>(tb, V, n, 32);
  __syncthreads();
  // Double-buffered stream of V blocks: block i is read from Vt[i & 1] while block i + 1 goes
  // into the other buffer and block i + 2 loads into registers; one barrier per block.
  for (int s0 = 0, i = 0; s0 < n; s0 += 32, ++i) {
    const f16v acc = tile<K>(a, Vt[i & 1], r, h);
    if (s0 + 32 < n) store_block<K>(Vt[(i + 1) & 1], tb);
    if (s0 + 64 < n) load_block<K>(tb, V, n, s0 + 64);
    const int sc = s0 + r;
    const bool colok = sc < n;
    const int scl = colok ? sc : n - 1;
    // past the last setting the key is NaN and never taken
    const float iw = colok ? 1.0f / (cap_c[scl] + cap_g[scl]) : __builtin_nanf("");
    if (P) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row0 + 8 * (v / 4) + 4 * h + (v % 4);
        if (colok && row < m) P[row * n + sc] = acc[v];
      }
    }
    // branch-free: greatest key p * iw among valid settings, the lane's settings in ascending
    // order, the first on ties
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float p = acc[v];
      const float key = p * iw;
      const bool better = p >= thr[v] && key > bK[v];
      bK[v] = better ? key : bK[v];
      bP[v] = better ? p : bP[v];
      bS[v] = better ? sc : bS[v];
    }
    __syncthreads();
  }
  // combine the 32 column lanes of each half-wave: greatest key, then lowest s
#pragma unroll
  for (int v = 0; v < 16; ++v) {
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) {
      const float K2 = __shfl_xor(bK[v], off, 64);
      const float P2 = __shfl_xor(bP[v], off, 64);
      const int S2 = __shfl_xor(bS[v], off, 64);
      const bool take = S2 >= 0 && (bS[v] < 0 || K2 > bK[v] || (K2 == bK[v] && S2 < bS[v]));
      bK[v] = take ? K2 : bK[v];
      bP[v] = take ? P2 : bP[v];
      bS[v] = take ? S2 : bS[v];
    }
  }
  if (r == 0) {
    const float ebase = cap_c[base] + cap_g[base];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = row0 + 8 * (v / 4) + 4 * h + (v % 4);
      if (row >= m) continue;
      const bool okb = pb[v] > 0.f && bS[v] >= 0;
      best_idx[row] = okb ? bS[v] : base;
      if (best_saving) {
        const int sb = okb ? bS[v] : base;
        const float E = (cap_c[sb] + cap_g[sb]) / bP[v];
        best_saving[row] = okb ? (ebase - E) / ebase : 0.f;
      }
      if (status) status[row] = okb ? OPEN_ROW_OK : OPEN_ROW_NONPOS_BASE;
    }
  }
}

}  // namespace openk

using namespace openk;

extern "C" open_status open_predict(open_ctx *ctx, const float *U, int64_t m, const float *V, int32_t n, int32_t k,
                                    float *P, const float *cap_cpu, const float *cap_gpu, int32_t base, float gamma,
                                    int32_t *best_idx, float *best_saving, int32_t *row_status) {
  if (!ctx) return OPEN_E_INVALID;
  if (!(k == 8 || k == 16 || k == 32 || k == 64)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (m < 0 || n <= 0 || base < 0 || base >= n) return fail(ctx, OPEN_E_INVALID, "bad shape or baseline index");
  if (!(gamma >= 0.0f) || !isfinite(gamma)) return fail(ctx, OPEN_E_INVALID, "gamma must be finite and >= 0");
  if (m > 0 && (!U || !V || !cap_cpu || !cap_gpu || !best_idx))
    return fail(ctx, OPEN_E_INVALID, "pointers must not be NULL");
  if (m == 0) return OPEN_OK;
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const dim3 grid((unsigned)((m + 127) / 128)), block(256);
  switch (k) {
    case 8:
      OPEN_LAUNCH(ctx, "predict_select_k8", k_predict_select<8>, grid, block, 0, U, m, V, n, cap_cpu, cap_gpu, base,
                  gamma, P, best_idx, best_saving, row_status);
      break;
    case 16:
      OPEN_LAUNCH(ctx, "predict_select_k16", k_predict_select<16>, grid, block, 0, U, m, V, n, cap_cpu, cap_gpu, base,
                  gamma, P, best_idx, best_saving, row_status);
      break;
    case 32:
      OPEN_LAUNCH(ctx, "predict_select_k32", k_predict_select<32>, grid, block, 0, U, m, V, n, cap_cpu, cap_gpu, base,
                  gamma, P, best_idx, best_saving, row_status);
      break;
    default:
      OPEN_LAUNCH(ctx, "predict_select_k64", k_predict_select<64>, grid, block, 0, U, m, V, n, cap_cpu, cap_gpu, base,
                  gamma, P, best_idx, best_saving, row_status);
      break;
  }
  return OPEN_OK;
}
