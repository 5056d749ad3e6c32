// Neural collaborative filtering fold-in (Section III-B.1 model, Section III-B.2 online
// imputation): each new application's embedding e is learned with the setting embeddings and
// the network frozen, by `steps` steps of gradient descent from e = 0 on
//   L(e) = (1/q) sum_j (y(e, s_j) - r_j)^2 + mu |e|^2,
//   y(e, s) = w3 . SELU(W2 SELU(W1 [e; s] + b1) + b2) + b3,   d = 32, 64 hidden units.
//
// The setting half of the first layer is the same for every application and every step, so
// a table C[j] = W1[:, d:] s_j + b1 (n x 64) is built once per call; a step then needs only
// a = W1[:, :d] e, and a setting's first pre-activation is a + C[j].
//
// One wavefront per application; lane l owns hidden unit l of both layers and lane k < 32 owns
// e_k.  Activations move between lanes with readlane (the index is a compile-time constant),
// W2 and the embedding half of W1 sit in LDS with an odd pitch so that both a row and a column
// are read without bank conflicts, and each lane keeps its row of W1[:, :d] in registers.
#include "common.h"

namespace openk {

constexpr int kNcfD = 32, kNcfH = 64;
constexpr int kNcfMaxSteps = 100000;  // bounds a launch's run time
constexpr int kNcfW2P = kNcfH + 1, kNcfW1P = kNcfD + 1;
constexpr float kSeluAlpha = 1.6732632423543772f, kSeluLambda = 1.0507009873554805f;

__device__ __forceinline__ void selu_and_grad(float z, float &h, float &dh) {
  if (z > 0.f) {
    h = kSeluLambda * z;
    dh = kSeluLambda;
  } else {
    const float ez = __expf(z);
    h = kSeluLambda * kSeluAlpha * (ez - 1.f);
    dh = kSeluLambda * kSeluAlpha * ez;
  }
}

__device__ __forceinline__ float wave_sum_f(float x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// C[j][l] = b1[l] + sum_k W1[l][d + k] S[j][k]
__global__ void k_ncf_table(const float *__restrict__ S, int n, const float *__restrict__ W1,
                            const float *__restrict__ b1, float *__restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kNcfH) return;
  const int j = (int)(t / kNcfH), l = (int)(t % kNcfH);
  float acc = b1[l];
  for (int k = 0; k < kNcfD; ++k) acc = __builtin_fmaf(W1[l * 2 * kNcfD + kNcfD + k], S[(int64_t)j * kNcfD + k], acc);
  C[t] = acc;
}

__global__ __launch_bounds__(256) void k_ncf_foldin(int64_t m, const int64_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ col, const float *__restrict__ val,
                                                    int n, const float *__restrict__ C, const float *__restrict__ W1,
                                                    const float *__restrict__ W2, const float *__restrict__ b2,
                                                    const float *__restrict__ w3, const float *__restrict__ b3,
                                                    int steps, float eta, float mu, float *__restrict__ E,
                                                    float *__restrict__ Lout, int32_t *__restrict__ status) {
  __shared__ float w2s[kNcfH * kNcfW2P];  // W2[m][k] at m * 65 + k
  __shared__ float w1s[kNcfH * kNcfW1P];  // W1[l][k], k < d, at l * 33 + k
  for (int q = threadIdx.x; q < kNcfH * kNcfH; q += blockDim.x) w2s[(q / kNcfH) * kNcfW2P + q % kNcfH] = W2[q];
  for (int q = threadIdx.x; q < kNcfH * kNcfD; q += blockDim.x)
    w1s[(q / kNcfD) * kNcfW1P + q % kNcfD] = W1[(q / kNcfD) * 2 * kNcfD + q % kNcfD];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  float w1r[kNcfD];  // this lane's row of W1[:, :d]
#pragma unroll
  for (int k = 0; k < kNcfD; ++k) w1r[k] = w1s[lane * kNcfW1P + k];
  const float b2l = b2[lane], w3l = w3[lane], bias3 = b3[0];

  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < m; i += nw) {
    const int64_t beg = ptr[i], end = ptr[i + 1];
    const int q = (int)(end - beg);
    // row checks: empty, setting index out of range, non-finite value
    int st = q <= 0 ? 1 : 0;
    if (st == 0) {
      bool bad_idx = false, bad_val = false;
      for (int64_t t = beg + lane; t < end; t += kWave) {
        const int j = col[t];
        bad_idx = bad_idx || j < 0 || j >= n;
        bad_val = bad_val || !__builtin_isfinite(val[t]);
      }
      if (__ballot(bad_idx)) st = 5;
      else if (__ballot(bad_val)) st = 3;
    }
    float e = 0.f;  // e_lane for lanes < 32
    float lossv = 0.f;
    if (st == 0) {
      const float inv_q = 1.f / (float)q;
      for (int it = 0; it <= steps; ++it) {
        // a_l = sum_k W1[l][k] e_k
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < kNcfD; ++k)
          a = __builtin_fmaf(w1r[k], __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, e), k)),
                             a);
        float g = 0.f, sq = 0.f;
        for (int64_t t = beg; t < end; ++t) {
          const int j = col[t];
          const float r = val[t];
          float h1, d1;
          selu_and_grad(a + C[(int64_t)j * kNcfH + lane], h1, d1);
          float z2 = b2l;
#pragma unroll
          for (int k = 0; k < kNcfH; ++k)
            z2 = __builtin_fmaf(w2s[lane * kNcfW2P + k],
                                __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, h1), k)), z2);
          float h2, d2;
          selu_and_grad(z2, h2, d2);
          const float y = wave_sum_f(w3l * h2) + bias3;
          const float res = y - r;
          sq = __builtin_fmaf(res, res, sq);
          if (it == steps) continue;  // the last pass only evaluates the loss
          const float dz2 = 2.f * res * inv_q * w3l * d2;
          float dh1 = 0.f;
#pragma unroll
          for (int mm = 0; mm < kNcfH; ++mm)
            dh1 = __builtin_fmaf(w2s[mm * kNcfW2P + lane],
                                 __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, dz2), mm)),
                                 dh1);
          g = __builtin_fmaf(dh1, d1, g);
        }
        if (it == steps) {
          const float ee = lane < kNcfD ? e * e : 0.f;
          lossv = sq * inv_q + mu * wave_sum_f(ee);
          break;
        }
        // de_k = sum_l W1[l][k] g_l + 2 mu e_k, on lanes k < d
        float de = 0.f;
        const int kk = lane < kNcfD ? lane : 0;
#pragma unroll
        for (int l = 0; l < kNcfH; ++l)
          de = __builtin_fmaf(w1s[l * kNcfW1P + kk],
                              __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, g), l)), de);
        if (lane < kNcfD) e -= eta * (de + 2.f * mu * e);
      }
    }
    if (lane < kNcfD) E[i * kNcfD + lane] = e;
    if (lane == 0) {
      if (Lout) Lout[i] = st == 0 ? lossv : 0.f;
      if (status) status[i] = st;
    }
  }
}

}  // namespace openk

using namespace openk;

extern "C" open_status open_ncf_foldin(open_ctx *ctx, const float *S, int32_t n, int32_t d, const float *W1,
                                       const float *b1, const float *W2, const float *b2, const float *w3,
                                       const float *b3, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                       const float *val, int32_t steps, float eta, float mu, float *E_out,
                                       float *loss_out, int32_t *row_status) {
  if (!ctx) return OPEN_E_INVALID;
  if (d != kNcfD) return fail(ctx, OPEN_E_UNSUPPORTED, "embedding width must be 32");
  if (n < 1 || m < 0 || steps < 0 || steps > kNcfMaxSteps || !(eta == eta) || !(mu == mu))
    return fail(ctx, OPEN_E_INVALID, "bad sizes, steps, eta or mu");
  if (m == 0) return OPEN_OK;
  if (!S || !W1 || !b1 || !W2 || !b2 || !w3 || !b3 || !row_ptr || !col || !val || !E_out)
    return fail(ctx, OPEN_E_INVALID, "null pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  void *tab = nullptr;
  open_status st;
  if ((st = ws_get(ctx, open_ctx::WS_NCF, sizeof(float) * (size_t)n * kNcfH, &tab))) return st;
  const int64_t tt = (int64_t)n * kNcfH;
  OPEN_LAUNCH(ctx, "ncf_table", k_ncf_table, dim3((unsigned)((tt + 255) / 256)), dim3(256), 0, S, n, W1, b1,
              (float *)tab);
  const int64_t cap = (int64_t)ctx->num_cu * 16;  // waves
  const int64_t waves = m < cap ? m : cap;
  OPEN_LAUNCH(ctx, "ncf_foldin", k_ncf_foldin, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, m, row_ptr, col, val,
              n, (const float *)tab, W1, W2, b2, w3, b3, steps, eta, mu, E_out, loss_out, row_status);
  return OPEN_OK;
}
