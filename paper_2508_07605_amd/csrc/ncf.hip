// Neural collaborative filtering fold-in (Section III-B.1 model, Section III-B.2 online
// imputation): each new application's embedding e is learned with the setting embeddings and
// the network frozen, by `steps` steps of gradient descent from e = 0 on
//   L(e) = (1/q) sum_j (y(e, s_j) - r_j)^2 + mu |e|^2,
//   y(e, s) = w3 . SELU(W2 SELU(W1 [e; s] + b1) + b2) + b3,   d = 32, 64 hidden units.
//
// The setting half of the first layer is the same for every application and every step, so
// a table C[j] = W1[:, d:] s_j + b1 (n x 64) is built once per call; a step then needs only
// a = W1[:, :d] e, and a setting's first pre-activation is a + C[j].
#include <math.h>

#include <new>

#include "common.h"
#include "dense.h"

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

// ---------------------------------------------------------------- offline training
// The model is trained on the dense offline matrix R (applications x settings, every entry
// observed) in batches of whole applications: batch entry b = g n + j pairs application
// apps[g] with setting j.  The products run through the shared BF16 MFMA GEMMs (SELU
// epilogues) and the batch-split weight gradients; the kernels here gather the inputs, form
// the loss and sum the embedding gradients in a fixed order.

// X[b] = [E[apps[g]] ; S[j]] (batch x 64)
__global__ void k_ncf_gather(int64_t B, int n, const int64_t *__restrict__ apps, const float *__restrict__ E,
                             const float *__restrict__ S, float *__restrict__ X) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < B * 2 * kNcfD;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / (2 * kNcfD);
    const int c = (int)(t % (2 * kNcfD));
    const int64_t g = b / n, j = b % n;
    X[t] = c < kNcfD ? E[apps[g] * kNcfD + c] : S[j * kNcfD + (c - kNcfD)];
  }
}

// dy[b] = 2 (y_b - r_b) / B, block partial sums of (y_b - r_b)^2 in float64
__global__ __launch_bounds__(256) void k_ncf_loss(int64_t B, int n, const float *__restrict__ y,
                                                  const int64_t *__restrict__ apps, const float *__restrict__ R,
                                                  float *__restrict__ dy, double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const float scale = 2.0f / (float)B;
  for (int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x; b < B; b += (int64_t)gridDim.x * 256) {
    const int64_t g = b / n, j = b % n;
    const float d = y[b] - R[apps[g] * n + j];
    dy[b] = scale * d;
    acc += (double)d * (double)d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < (unsigned)s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// gE[apps[g]] = sum_j dX[g n + j][0 .. 32) (j in order), gS[j] = sum_g dX[g n + j][32 .. 64)
// (g in order); the batch's applications are distinct and gE is zero elsewhere
__global__ void k_ncf_emb_grad(int G, int n, const int64_t *__restrict__ apps, const float *__restrict__ dX,
                               float *__restrict__ gE, float *__restrict__ gS) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nE = (int64_t)G * kNcfD, nS = (int64_t)n * kNcfD;
  if (t < nE) {
    const int64_t g = t / kNcfD;
    const int c = (int)(t % kNcfD);
    float acc = 0.f;
    for (int j = 0; j < n; ++j) acc += dX[(g * n + j) * 2 * kNcfD + c];
    gE[apps[g] * kNcfD + c] = acc;
  } else if (t < nE + nS) {
    const int64_t j = (t - nE) / kNcfD;
    const int c = (int)((t - nE) % kNcfD);
    float acc = 0.f;
    for (int g = 0; g < G; ++g) acc += dX[((int64_t)g * n + j) * 2 * kNcfD + kNcfD + c];
    gS[j * kNcfD + c] = acc;
  }
}

constexpr int kNcfLossBlocks = 256;

// Parameter packing of the trained model (float32): E (m_off x d), S (n x d), W1 (H x 2d),
// b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1).
struct NcfLayout {
  int64_t E, S, W1, b1, W2, b2, w3, b3, total;
  NcfLayout(int64_t m_off, int64_t n) {
    E = 0;
    S = E + m_off * kNcfD;
    W1 = S + n * kNcfD;
    b1 = W1 + (int64_t)kNcfH * 2 * kNcfD;
    W2 = b1 + kNcfH;
    b2 = W2 + (int64_t)kNcfH * kNcfH;
    w3 = b2 + kNcfH;
    b3 = w3 + kNcfH;
    total = b3 + 1;
  }
};

// Device buffers of one training call.
struct NcfTrainBufs {
  int64_t B = 0;
  float *X = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *y = nullptr, *dy = nullptr;
  float *dZ2 = nullptr, *dZ1 = nullptr, *dX = nullptr, *part = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;
  double *lpart = nullptr, *loss = nullptr;
  TrainState *st = nullptr;
  void release() {
    float *fs[] = {X, Z1, H1, Z2, H2, y, dy, dZ2, dZ1, dX, part, g, am, av};
    for (float *f : fs) (void)hipFree(f);
    (void)hipFree(lpart);
    (void)hipFree(loss);
    (void)hipFree(st);
  }
  bool alloc(int64_t Bsz, int64_t np) {
    B = Bsz;
    const size_t a = sizeof(float) * (size_t)Bsz * 2 * kNcfD;
    int64_t wp = dense_wgrad_part_floats(Bsz, kNcfH, kNcfH);
    if (dense_wgrad_part_floats(Bsz, kNcfH, 2 * kNcfD) > wp) wp = dense_wgrad_part_floats(Bsz, kNcfH, 2 * kNcfD);
    if (dense_wgrad_part_floats(Bsz, 1, kNcfH) > wp) wp = dense_wgrad_part_floats(Bsz, 1, kNcfH);
    const bool ok = !hipMalloc(&X, a) && !hipMalloc(&Z1, a) && !hipMalloc(&H1, a) && !hipMalloc(&Z2, a) &&
                    !hipMalloc(&H2, a) && !hipMalloc(&y, sizeof(float) * Bsz) && !hipMalloc(&dy, sizeof(float) * Bsz) &&
                    !hipMalloc(&dZ2, a) && !hipMalloc(&dZ1, a) && !hipMalloc(&dX, a) &&
                    !hipMalloc(&part, sizeof(float) * (size_t)wp) && !hipMalloc(&g, sizeof(float) * (size_t)np) &&
                    !hipMalloc(&am, sizeof(float) * (size_t)np) && !hipMalloc(&av, sizeof(float) * (size_t)np) &&
                    !hipMalloc(&lpart, sizeof(double) * (kNcfLossBlocks + 8)) && !hipMalloc(&loss, sizeof(double) * 8) &&
                    !hipMalloc(&st, sizeof(TrainState));
    if (!ok) (void)hipGetLastError();
    return ok;
  }
};

// Loss and gradient of one batch of G applications (their indices in `apps`, on the device)
// into b.g; the loss to b.loss and, when given, to loss_steps[t].
static open_status ncf_batch_grad(open_ctx *ctx, const NcfLayout &L, int n, const float *R, const float *P,
                                  const int64_t *apps, int G, NcfTrainBufs &b, float *loss_steps) {
  const int64_t B = (int64_t)G * n;
  const int D2 = 2 * kNcfD, H = kNcfH;
  open_status st;
  int64_t blocks = (B * D2 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  OPEN_LAUNCH(ctx, "ncf_gather", k_ncf_gather, dim3((unsigned)blocks), dim3(256), 0, B, n, apps, P + L.E, P + L.S,
              b.X);
  // forward: Z1 = X W1^T + b1, H1 = SELU(Z1); Z2 = H1 W2^T + b2, H2 = SELU(Z2); y = H2 w3 + b3
  if ((st = dense_gemm(ctx, "ncf_gemm_l1", EPI_BIAS_SELU, (int)B, H, D2, b.X, D2, 1, P + L.W1, D2, 1, b.H1, H,
                       P + L.b1, b.Z1, H)))
    return st;
  if ((st = dense_gemm(ctx, "ncf_gemm_l2", EPI_BIAS_SELU, (int)B, H, H, b.H1, H, 1, P + L.W2, H, 1, b.H2, H, P + L.b2,
                       b.Z2, H)))
    return st;
  if ((st = dense_gemm(ctx, "ncf_gemm_out", EPI_BIAS, (int)B, 1, H, b.H2, H, 1, P + L.w3, H, 1, b.y, 1, P + L.b3)))
    return st;
  OPEN_LAUNCH(ctx, "ncf_loss", k_ncf_loss, dim3(kNcfLossBlocks), dim3(256), 0, B, n, b.y, apps, R, b.dy, b.lpart);
  if ((st = dense_loss_final(ctx, b.lpart, kNcfLossBlocks, B, b.loss, nullptr, b.st, loss_steps))) return st;
  // backward
  float *g = b.g;
  if ((st = dense_wgrad(ctx, "ncf_wgrad_out", 1, H, B, b.dy, b.H2, b.part, g + L.w3))) return st;  // w3, b3
  // dZ2 = (dy w3^T) * SELU'(Z2)
  if ((st = dense_gemm(ctx, "ncf_gemm_dz2", EPI_SELU_GRAD, (int)B, H, 1, b.dy, 1, 1, P + L.w3, 1, 1, b.dZ2, H, nullptr,
                       b.Z2, H)))
    return st;
  if ((st = dense_wgrad(ctx, "ncf_wgrad_l2", H, H, B, b.dZ2, b.H1, b.part, g + L.W2))) return st;  // W2, b2
  // dZ1 = (dZ2 W2) * SELU'(Z1)
  if ((st = dense_gemm(ctx, "ncf_gemm_dz1", EPI_SELU_GRAD, (int)B, H, H, b.dZ2, H, 1, P + L.W2, 1, H, b.dZ1, H, nullptr,
                       b.Z1, H)))
    return st;
  if ((st = dense_wgrad(ctx, "ncf_wgrad_l1", H, D2, B, b.dZ1, b.X, b.part, g + L.W1))) return st;  // W1, b1
  // dX = dZ1 W1, then the embedding gradients
  if ((st = dense_gemm(ctx, "ncf_gemm_dx", EPI_STORE, (int)B, D2, H, b.dZ1, H, 1, P + L.W1, 1, D2, b.dX, D2)))
    return st;
  const int64_t nE = L.S - L.E;
  OPEN_LAUNCH(ctx, "fill", k_fill_i32, dim3(256), dim3(256), 0, (int *)(g + L.E), nE, 0);
  const int64_t th = ((int64_t)G + n) * kNcfD;
  OPEN_LAUNCH(ctx, "ncf_emb_grad", k_ncf_emb_grad, dim3((unsigned)((th + 255) / 256)), dim3(256), 0, G, n, apps, b.dX,
              g + L.E, g + L.S);
  return OPEN_OK;
}

constexpr int64_t kNcfMaxBatch = int64_t(1) << 20;  // batch entries (applications x settings)

static open_status ncf_train_check(open_ctx *ctx, int64_t m_off, int32_t n, int32_t d, const float *R,
                                   const float *params, int64_t G) {
  if (d != kNcfD) return fail(ctx, OPEN_E_UNSUPPORTED, "embedding width must be 32");
  if (m_off < 1 || n < 1 || m_off > INT32_MAX) return fail(ctx, OPEN_E_INVALID, "bad matrix shape");
  if (!R || !params) return fail(ctx, OPEN_E_INVALID, "null pointer");
  if (G < 1 || G > m_off || G * n > kNcfMaxBatch)
    return fail(ctx, OPEN_E_INVALID, "applications per batch must be in [1, m_off] with at most 2^20 entries");
  return OPEN_OK;
}

}  // namespace openk

using namespace openk;

extern "C" int64_t open_ncf_num_params(int64_t m_off, int32_t n) { return NcfLayout(m_off, n).total; }

extern "C" open_status open_ncf_loss_grad(open_ctx *ctx, int64_t m_off, int32_t n, int32_t d, const float *R,
                                          const float *params, const int64_t *apps, int32_t G, double *loss,
                                          float *grads_host) {
  if (!ctx) return OPEN_E_INVALID;
  open_status st = ncf_train_check(ctx, m_off, n, d, R, params, G);
  if (st) return st;
  if (!apps || !loss || !grads_host) return fail(ctx, OPEN_E_INVALID, "null pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const NcfLayout L(m_off, n);
  NcfTrainBufs b;
  if (!b.alloc((int64_t)G * n, L.total)) {
    b.release();
    return fail(ctx, OPEN_E_NOMEM, "NCF training buffers");
  }
  st = dense_train_state_reset(ctx, b.st);
  if (!st) st = ncf_batch_grad(ctx, L, n, R, params, apps, G, b, nullptr);
  double *h = nullptr;
  if (!st) st = pinned_get(ctx, 64, (void **)&h);
  if (!st && (hipMemcpyAsync(grads_host, b.g, sizeof(float) * L.total, hipMemcpyDeviceToHost, ctx->stream) ||
              hipMemcpyAsync(h, b.loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream) ||
              hipStreamSynchronize(ctx->stream)))
    st = fail(ctx, OPEN_E_DEVICE, "reading the gradient");
  if (!st) *loss = h[0];
  (void)hipStreamSynchronize(ctx->stream);
  b.release();
  return st;
}

extern "C" open_status open_ncf_train(open_ctx *ctx, int64_t m_off, int32_t n, int32_t d, const float *R,
                                      float *params, int32_t apps_per_batch, float lr, int32_t epochs, uint64_t seed,
                                      float *loss_hist) {
  if (!ctx) return OPEN_E_INVALID;
  open_status st = ncf_train_check(ctx, m_off, n, d, R, params, apps_per_batch);
  if (st) return st;
  if (epochs < 0 || !(lr > 0.f) || !isfinite(lr)) return fail(ctx, OPEN_E_INVALID, "bad epochs or learning rate");
  if (epochs == 0) return OPEN_OK;
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const NcfLayout L(m_off, n);
  const int G = apps_per_batch;
  const int64_t spe = m_off / G, total = spe * epochs;
  NcfTrainBufs b;
  int64_t *perm = nullptr, *rows = nullptr;
  float *losses = nullptr;
  if (!b.alloc((int64_t)G * n, L.total) || hipMalloc(&perm, sizeof(int64_t) * m_off) ||
      hipMalloc(&rows, sizeof(int64_t) * G) || hipMalloc(&losses, sizeof(float) * total)) {
    (void)hipGetLastError();
    b.release();
    (void)hipFree(perm);
    (void)hipFree(rows);
    (void)hipFree(losses);
    return fail(ctx, OPEN_E_NOMEM, "NCF training buffers");
  }
  OPEN_LAUNCH(ctx, "fill", k_fill_i32, dim3(256), dim3(256), 0, (int *)b.am, L.total, 0);
  OPEN_LAUNCH(ctx, "fill", k_fill_i32, dim3(256), dim3(256), 0, (int *)b.av, L.total, 0);
  st = dense_train_state_reset(ctx, b.st);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto one_step = [&]() -> open_status {
    open_status e;
    if ((e = dense_rows_of_step(ctx, perm, G, b.st, rows))) return e;
    if ((e = ncf_batch_grad(ctx, L, n, R, params, rows, G, b, losses))) return e;
    return dense_adam_step(ctx, L.total, params, b.g, b.am, b.av, lr, b.st);
  };
  for (int32_t e = 0; e < epochs && st == OPEN_OK; ++e) {
    if ((st = dense_shuffle(ctx, m_off, seed, e, perm, b.st))) break;
    for (int64_t s = 0; s < spe && st == OPEN_OK; ++s) {
      if (!exec) {
        if ((st = one_step())) break;  // the first step runs eagerly, the next one is recorded
        if (s + 1 < spe || e + 1 < epochs) {
          if ((st = graph_capture(ctx, one_step, &graph))) break;
          if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(ctx, OPEN_E_DEVICE, "graph instantiation failed");
          }
        }
        continue;
      }
      if (hipGraphLaunch(exec, ctx->stream) != hipSuccess) st = fail(ctx, OPEN_E_DEVICE, "graph launch failed");
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (st == OPEN_OK && loss_hist) {
    float *hl = new (std::nothrow) float[(size_t)total];
    if (!hl) {
      st = fail(ctx, OPEN_E_NOMEM, "loss history");
    } else {
      if (hipMemcpyAsync(hl, losses, sizeof(float) * (size_t)total, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess) {
        st = fail(ctx, OPEN_E_DEVICE, "reading the losses");
      } else {
        for (int32_t e = 0; e < epochs; ++e) {
          double sum = 0.0;
          for (int64_t s = 0; s < spe; ++s) sum += hl[e * spe + s];
          loss_hist[e] = (float)(sum / (double)spe);
        }
      }
      delete[] hl;
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  b.release();
  (void)hipFree(perm);
  (void)hipFree(rows);
  (void)hipFree(losses);
  return st;
}

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
