// Fused prediction + energy-efficient cap selection (Algorithm 2, Section III-B.3).
//
// p_is = u_i . v_s is formed tile by tile on FP32 MFMA (v_mfma_f32_32x32x2_f32): a wavefront
// owns 32 rows, keeps their factor rows in registers (A operand) and streams the setting
// factors through LDS in blocks of 32 settings (B operand, stored transposed with a padded
// stride so the 32 lanes of a half-wave read distinct banks).  The epilogue applies the
// paper's rule to every element without materialising p:
//   p_base = p_ib                          (the same MFMA value the scan sees for s = b)
//   valid  = p > 0  and  1 - p / p_base <= gamma      (float32, correctly rounded division)
//   E      = (c_s + g_s) / p                (float32)
//   keep the least E, the lowest s on ties  ==  the greatest saving (E_base - E) / E_base
// Each lane scans its own settings in ascending order; the 32 lanes of a half-wave are then
// combined by (E, s) in a butterfly.  The full prediction P is written only when asked.
#include <math.h>

#include "common.h"

namespace openk {

typedef float f16v __attribute__((ext_vector_type(16)));

template <int K>
__device__ __forceinline__ void stage_block(float *Vt, const float *__restrict__ V, int n, int s0) {
  constexpr int LD = 33;
  for (int e = threadIdx.x; e < 32 * K; e += blockDim.x) {
    const int j = e / K, kk = e % K;
    Vt[kk * LD + j] = (s0 + j < n) ? V[(int64_t)(s0 + j) * K + kk] : 0.f;
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

template <int K>
__global__ __launch_bounds__(256) void k_predict_select(const float *__restrict__ U, int64_t m,
                                                        const float *__restrict__ V, int n,
                                                        const float *__restrict__ cap_c,
                                                        const float *__restrict__ cap_g, int base, float gamma,
                                                        float *__restrict__ P, int32_t *__restrict__ best_idx,
                                                        float *__restrict__ best_saving,
                                                        int32_t *__restrict__ status) {
  constexpr int H = K / 2, LD = 33;
  __shared__ float Vt[K * LD];
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
  stage_block<K>(Vt, V, n, sb0);
  __syncthreads();
  float pb[16];
  {
    const f16v acc = tile<K>(a, Vt, r, h);
#pragma unroll
    for (int v = 0; v < 16; ++v) pb[v] = __shfl(acc[v], jb + 32 * h, 64);
  }
  float bE[16];
  int bS[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    bE[v] = 0.f;
    bS[v] = -1;
  }
  for (int s0 = 0; s0 < n; s0 += 32) {
    __syncthreads();
    stage_block<K>(Vt, V, n, s0);
    __syncthreads();
    const f16v acc = tile<K>(a, Vt, r, h);
    const int sc = s0 + r;
    const bool colok = sc < n;
    const float wcol = colok ? cap_c[sc] + cap_g[sc] : 0.f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = row0 + 8 * (v / 4) + 4 * h + (v % 4);
      const float p = acc[v];
      if (P && colok && row < m) P[row * n + sc] = p;
      const bool valid = colok && p > 0.f && pb[v] > 0.f && (1.0f - p / pb[v]) <= gamma;
      if (valid) {
        const float E = wcol / p;
        if (bS[v] < 0 || E < bE[v]) {
          bE[v] = E;
          bS[v] = sc;
        }
      }
    }
  }
  // combine the 32 column lanes of each half-wave: least E, then lowest s
#pragma unroll
  for (int v = 0; v < 16; ++v) {
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) {
      const float E2 = __shfl_xor(bE[v], off, 64);
      const int S2 = __shfl_xor(bS[v], off, 64);
      const bool take = S2 >= 0 && (bS[v] < 0 || E2 < bE[v] || (E2 == bE[v] && S2 < bS[v]));
      bE[v] = take ? E2 : bE[v];
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
      if (best_saving) best_saving[row] = okb ? (ebase - bE[v]) / ebase : 0.f;
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
