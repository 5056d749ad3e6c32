// Neural collaborative filtering fold-in (Section III-B.1 model, Section III-B.2 online
// imputation): each new application's embedding e is learned with the setting embeddings and
// the network frozen, by `steps` steps of gradient descent from e = 0 on
//   L(e) = (1/q) sum_j (y(e, s_j) - r_j)^2 + mu |e|^2,
//   y(e, s) = w3 . SELU(W2 SELU(W1 [e; s] + b1) + b2) + b3,   d = 32, 64 hidden units.
//
// The setting half of the first layer is the same for every application and every step, so
// a table C[j] = W1[:, d:] s_j + b1 (n x 64) is built once per call; a step then needs only
// a = W1[:, :d] e, and a setting's first pre-activation is a + C[j].
#include "common.h"

namespace openk {

constexpr int kNcfD = 32, kNcfH = 64;
constexpr int kNcfMaxSteps = 100000;  // bounds a launch's run time
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

// Observation tiles on FP32 MFMA (v_mfma_f32_32x32x2f32).  One wavefront per two applications:
// the 32 MFMA columns hold 16 observations of each (lane j = l % 32 is column j, g = l / 32 the
// half); the MFMA keeps columns apart, so each column simply carries its own application's
// embedding.  Every 32 x 32 result holds, in register v of lane (j, g),
// row 8 (v/4) + 4 g + v%4 of its block; hidden unit U(b, v, g) = 32 b + that row, embedding
// index K(v, g) = that row.  Each product's contraction index is ordered so that its B operand
// is a register the lane already holds:
//   a   = W1e e         (64 x 32):  step s, half g <-> embedding K(s, g)   (e kept as e[K(v, g)])
//   Z2  = W2 H1         (64 x 64):  step t, half g <-> hidden U(t/16, t%16, g)
//   dH1 = W2^T dZ2      (64 x 64):  step t, half g <-> layer-2 unit U(t/16, t%16, g)
//   DE  = W1e^T dZ1     (32 x 64):  step t, half g <-> hidden U(t/16, t%16, g)
// so activations never move between lanes.  The A operands depend on the lane only and sit in
// LDS once per block, slot-major so that consecutive lanes read consecutive 16-byte words.
// DE's columns (observations) are summed across each application's 16 lanes of a half.
constexpr int kNcfTA = 0, kNcfTF = 8, kNcfTB = 24, kNcfTE = 40, kNcfTW3 = 48, kNcfTB2 = 56, kNcfTSlots = 64;

__device__ __forceinline__ f16 mfma32(float a, float b, f16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int ncf_row(int v, int g) { return 8 * (v >> 2) + 4 * g + (v & 3); }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_ncf_foldin(int64_t m, const RowRef *__restrict__ list,
                                                    const int32_t *__restrict__ col, const float *__restrict__ val,
                                                    int n, const float *__restrict__ C, const float *__restrict__ W1,
                                                    const float *__restrict__ W2, const float *__restrict__ b2,
                                                    const float *__restrict__ w3, const float *__restrict__ b3,
                                                    int steps, float eta, float mu, float *__restrict__ E,
                                                    float *__restrict__ Lout, int32_t *__restrict__ status) {
  // tab[slot][lane]: per-lane operands, four floats per slot
  __shared__ f4 tab[kNcfTSlots][kWave];
  if (threadIdx.x < kWave) {
    const int l = threadIdx.x, j = l & 31, g = l >> 5;
    float *t = nullptr;
    // a = W1e e: A[b][s] = W1e[32 b + j][K(s, g)]
    for (int b = 0; b < 2; ++b)
      for (int s = 0; s < 16; ++s) {
        t = reinterpret_cast<float *>(&tab[kNcfTA + (16 * b + s) / 4][l]);
        t[s & 3] = W1[(32 * b + j) * 2 * kNcfD + ncf_row(s, g)];
      }
    // Z2 = W2 H1: A[ob][t] = W2[32 ob + j][U(t)], and dH1 = W2^T dZ2: A[b][t] = W2[U(t)][32 b + j]
    for (int ob = 0; ob < 2; ++ob)
      for (int q = 0; q < 32; ++q) {
        const int u = 32 * (q >> 4) + ncf_row(q & 15, g);
        reinterpret_cast<float *>(&tab[kNcfTF + (32 * ob + q) / 4][l])[q & 3] = W2[(32 * ob + j) * kNcfH + u];
        reinterpret_cast<float *>(&tab[kNcfTB + (32 * ob + q) / 4][l])[q & 3] = W2[u * kNcfH + 32 * ob + j];
      }
    // DE = W1e^T dZ1: A[t] = W1e[U(t)][j]
    for (int q = 0; q < 32; ++q) {
      const int u = 32 * (q >> 4) + ncf_row(q & 15, g);
      reinterpret_cast<float *>(&tab[kNcfTE + q / 4][l])[q & 3] = W1[u * 2 * kNcfD + j];
    }
    // w3 and b2 at this lane's rows
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 16; ++v) {
        const int u = 32 * b + ncf_row(v, g);
        reinterpret_cast<float *>(&tab[kNcfTW3 + (16 * b + v) / 4][l])[v & 3] = w3[u];
        reinterpret_cast<float *>(&tab[kNcfTB2 + (16 * b + v) / 4][l])[v & 3] = b2[u];
      }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, jl = lane & 31, g = lane >> 5;
  const float bias3 = b3[0];
  // The table reads go through an offset the compiler cannot see through, renewed every tile,
  // so that it reads the operands from LDS where they are used instead of holding all 256 in
  // registers.
  int toff = 0;
  auto T = [&](int slot, int q) {
    return reinterpret_cast<const float *>(&tab[0][0])[((slot + q / 4) * kWave + lane + toff) * 4 + (q & 3)];
  };

  // two applications per wavefront: columns 0..15 of every tile belong to the first, 16..31
  // to the second (observations in tiles of 16 per application)
  const int half = jl >> 4, jc = jl & 15;
  const uint64_t appmask = 0x0000ffff0000ffffull << (16 * half);
  const int64_t npairs = (m + 1) >> 1;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t pr = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); pr < npairs; pr += nw) {
    const int64_t li = 2 * pr + half;  // this lane's application: entry li of the size-ordered list
    const bool has = li < m;
    const RowRef rec = has ? list[li] : RowRef{0, 0, 0};
    const int64_t i = rec.row, beg = rec.beg, end = rec.beg + rec.cnt;
    const int q = rec.cnt;
    int st = q <= 0 ? 1 : 0;
    {
      bool bad_idx = false, bad_val = false;
      for (int64_t t = beg + jc + 16 * g; st == 0 && t < end; t += 32) {
        const int j = col[t];
        bad_idx = bad_idx || j < 0 || j >= n;
        bad_val = bad_val || !__builtin_isfinite(val[t]);
      }
      if (st == 0 && (__ballot(bad_idx) & appmask)) st = 5;
      else if (st == 0 && (__ballot(bad_val) & appmask)) st = 3;
    }
    const bool live = has && st == 0;
    float e[16];  // e[v] = embedding K(v, g) of this lane's application
#pragma unroll
    for (int v = 0; v < 16; ++v) e[v] = 0.f;
    float lossv = 0.f;
    const int qt = live ? (q + 15) >> 4 : 0;
    const int ntiles = max(qt, __shfl_xor(qt, 16, kWave));  // the same in every lane
    if (ntiles > 0) {
      const float inv_q = live ? 1.f / (float)q : 0.f;
      for (int it = 0; it <= steps; ++it) {
        // a at this lane's hidden units
        asm volatile("" : "+v"(toff));
        f16 a[2] = {};
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int s2 = 0; s2 < 16; ++s2) a[b] = mfma32(T(kNcfTA, 16 * b + s2), e[s2], a[b]);
        f16 de = {};
        float sq = 0.f;
        for (int tt = 0; tt < ntiles; ++tt) {
          asm volatile("" : "+v"(toff));
          const int64_t t = beg + 16 * tt + jc;
          const bool valid = live && t < end;
          const float *crow = C + (int64_t)(valid ? col[t] : 0) * kNcfH;
          const float r = valid ? val[t] : 0.f;
          // forward: Z2 = b2 + W2 SELU(a + c)
          f16 z2[2];
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) z2[b][v] = T(kNcfTB2, 16 * b + v);
          float cz[32];
#pragma unroll
          for (int q2 = 0; q2 < 32; ++q2) cz[q2] = crow[32 * (q2 >> 4) + ncf_row(q2 & 15, g)];
#pragma unroll
          for (int q2 = 0; q2 < 32; ++q2) {
            float h1;
            selu_and_grad(a[q2 >> 4][q2 & 15] + cz[q2], h1, cz[q2]);  // cz now holds SELU'(z1)
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) z2[ob] = mfma32(T(kNcfTF, 32 * ob + q2), h1, z2[ob]);
          }
          // output and residual of this column's observation (each half holds half of the sum)
          float yp = 0.f;
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              float h2, d2;
              selu_and_grad(z2[b][v], h2, d2);
              yp = __builtin_fmaf(T(kNcfTW3, 16 * b + v), h2, yp);
            }
          const float y = yp + __shfl_xor(yp, 32, kWave) + bias3;
          const float res = valid ? y - r : 0.f;
          sq = __builtin_fmaf(res, res, sq);
          if (it == steps) continue;  // the last pass only evaluates the loss
          // backward: dH1 = W2^T dZ2, dZ2 = (2 res / q) w3 SELU'(z2)
          const float dy = 2.f * res * inv_q;
          f16 dh1[2] = {};
#pragma unroll
          for (int q2 = 0; q2 < 32; ++q2) {
            float h2, d2;
            selu_and_grad(z2[q2 >> 4][q2 & 15], h2, d2);
            const float dz2 = dy * T(kNcfTW3, q2) * d2;
#pragma unroll
            for (int b = 0; b < 2; ++b) dh1[b] = mfma32(T(kNcfTB, 32 * b + q2), dz2, dh1[b]);
          }
          // DE += W1e^T (dH1 * SELU'(a + c))
#pragma unroll
          for (int q2 = 0; q2 < 32; ++q2) de = mfma32(T(kNcfTE, q2), dh1[q2 >> 4][q2 & 15] * cz[q2], de);
        }
        if (it == steps) {
          float ee = 0.f;
#pragma unroll
          for (int v = 0; v < 16; ++v) ee = __builtin_fmaf(e[v], e[v], ee);
          // squared residuals: one per column in each half; embedding: each half holds 16 indices
          float sqt = g == 0 ? sq : 0.f;
#pragma unroll
          for (int off = 1; off < 16; off <<= 1) sqt += __shfl_xor(sqt, off, kWave);
          lossv = sqt * inv_q + mu * (ee + __shfl_xor(ee, 32, kWave));
          break;
        }
        // sum DE over the application's 16 columns, then the step
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float x = de[v];
#pragma unroll
          for (int off = 1; off < 16; off <<= 1) x += __shfl_xor(x, off, kWave);
          if (live) e[v] -= eta * (x + 2.f * mu * e[v]);
        }
      }
    }
    if (has && jc == 0) {
#pragma unroll
      for (int v = 0; v < 16; ++v) E[i * kNcfD + ncf_row(v, g)] = e[v];
      if (g == 0) {
        if (Lout) Lout[i] = live ? lossv : 0.f;
        if (status) status[i] = st;
      }
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
  if (m > INT32_MAX) return fail(ctx, OPEN_E_UNSUPPORTED, "more than 2^31 - 1 rows");
  if (!S || !W1 || !b1 || !W2 || !b2 || !w3 || !b3 || !row_ptr || !col || !val || !E_out)
    return fail(ctx, OPEN_E_INVALID, "null pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  void *tab = nullptr;
  open_status st;
  if ((st = ws_get(ctx, open_ctx::WS_NCF, sizeof(float) * (size_t)n * kNcfH, &tab))) return st;
  const int64_t tt = (int64_t)n * kNcfH;
  OPEN_LAUNCH(ctx, "ncf_table", k_ncf_table, dim3((unsigned)((tt + 255) / 256)), dim3(256), 0, S, n, W1, b1,
              (float *)tab);
  // applications in order of observed count, so that the two of a wavefront need about as
  // many observation tiles
  RowRef *list = nullptr;
  int64_t *cls = nullptr;
  if ((st = bucket_rows(ctx, m, row_ptr, kNcfD, &list, &cls, kSplitMin))) return st;
  const int64_t cap = (int64_t)ctx->num_cu * 16;  // waves
  const int64_t pairs = (m + 1) / 2;  // two applications per wavefront
  const int64_t waves = pairs < cap ? pairs : cap;
  OPEN_LAUNCH(ctx, "ncf_foldin", k_ncf_foldin, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, m,
              (const RowRef *)list, col, val, n, (const float *)tab, W1, W2, b2, w3, b3, steps, eta, mu, E_out,
              loss_out, row_status);
  return OPEN_OK;
}
