// Fold-in surrogate network: training and inference.
//
//   x  = [r * mask ; mask]                      (length 2n, never materialised)
//   z1 = W1 x + b1 = b1 + sum_{j in O} (r_j W1[:, j] + W1[:, n + j])    sparse first layer
//   h1 = GELU(z1);  z2 = W2 h1 + b2;  h2 = GELU(z2);  u = W3 h2 + b3
//   GELU(z) = z/2 (1 + erf(z / sqrt 2))
//
// Weights live as float32 masters (updated by Adam) and as bfloat16 copies (round to
// nearest even) for the products.  The sparse first layer accumulates value x weight in
// float32 from a transposed bfloat16 copy of W1 (one contiguous hidden vector per input
// feature).  The dense products run on BF16 MFMA (v_mfma_f32_32x32x16_bf16) with float32
// accumulation through one tiled GEMM kernel whose epilogue adds the bias and applies GELU,
// or multiplies by GELU'(z) in the backward pass.  The sparse W1 gradient is accumulated per
// input feature over a column view of the batch, in a fixed order (no float atomics).
#include <math.h>
#include <string.h>

#include <new>

#include "common.h"

namespace openk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// float32 -> bfloat16 bits, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, formula 7.1.26 (absolute
// error below 1.5e-7, under the float32 rounding of the activations):
//   erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),  t = 1 / (1 + p x),  x >= 0
// and erf(-x) = -erf(x).  One reciprocal and one exponential instead of the library's erff.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = __builtin_fabsf(x);
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, ax, 1.0f));
  float q = __builtin_fmaf(t, 1.061405429f, -1.453152027f);
  q = __builtin_fmaf(t, q, 1.421413741f);
  q = __builtin_fmaf(t, q, -0.284496736f);
  q = __builtin_fmaf(t, q, 0.254829592f);
  const float e = __expf(-ax * ax);
  return __builtin_copysignf(__builtin_fmaf(-t * q, e, 1.0f), x);
}
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// ---------------------------------------------------------------- bfloat16 weight copies
// W1T[j][h] = bf16(W1[h][j]) (2n x H);  Wb[i] = bf16(W[i]) for W2 and W3 (row-major as given)
__global__ void k_pack_w1t(const float *__restrict__ W1, int H, int twon, uint16_t *__restrict__ W1T) {
  const int64_t total = (int64_t)H * twon;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / H, h = e % H;
    W1T[e] = f2bf(W1[h * twon + j]);
  }
}

// ---------------------------------------------------------------- sparse first layer
// One wavefront per batch row, lane l owns hidden units 4l..4l+3 (H = 256).
// rows (nullable) maps batch index b -> CSR row.  Writes z1 (nullable) and h1 = GELU(z1).
__global__ __launch_bounds__(256) void k_layer1(int64_t B, const int64_t *__restrict__ rows,
                                                const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                const float *__restrict__ val, int n,
                                                const uint16_t *__restrict__ W1T, const float *__restrict__ b1,
                                                float *__restrict__ z1, float *__restrict__ h1) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < B; b += nw) {
    const int64_t i = rows ? rows[b] : b;
    f4 z = *reinterpret_cast<const f4 *>(b1 + 4 * lane);
    for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t) {
      const int j = col[t];
      if (j < 0 || j >= n) continue;
      const float r = val[t];
      const uint2 wa = *reinterpret_cast<const uint2 *>(W1T + (int64_t)j * 256 + 4 * lane);
      const uint2 wm = *reinterpret_cast<const uint2 *>(W1T + (int64_t)(n + j) * 256 + 4 * lane);
      z[0] += __builtin_fmaf(r, bf2f((uint16_t)(wa.x & 0xffff)), bf2f((uint16_t)(wm.x & 0xffff)));
      z[1] += __builtin_fmaf(r, bf2f((uint16_t)(wa.x >> 16)), bf2f((uint16_t)(wm.x >> 16)));
      z[2] += __builtin_fmaf(r, bf2f((uint16_t)(wa.y & 0xffff)), bf2f((uint16_t)(wm.y & 0xffff)));
      z[3] += __builtin_fmaf(r, bf2f((uint16_t)(wa.y >> 16)), bf2f((uint16_t)(wm.y >> 16)));
    }
    if (z1) *reinterpret_cast<f4 *>(z1 + b * 256 + 4 * lane) = z;
    f4 hv;
    hv[0] = gelu(z[0]);
    hv[1] = gelu(z[1]);
    hv[2] = gelu(z[2]);
    hv[3] = gelu(z[3]);
    *reinterpret_cast<f4 *>(h1 + b * 256 + 4 * lane) = hv;
  }
}

// ---------------------------------------------------------------- tiled BF16 MFMA GEMM
// C[m][n] = sum_k A(m, k) B(n, k), A(m, k) = A[m*sam + k*sak], B(n, k) = B[n*sbn + k*sbk],
// float32 operands rounded to bfloat16 when staged in LDS, float32 accumulation.
// Block tile 64 x 64, four wavefronts of 32 x 32 (v_mfma_f32_32x32x16_bf16), K chunks of 32.
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int Kd, const float *__restrict__ A, int64_t sam,
                                              int64_t sak, const float *__restrict__ Bm, int64_t sbn, int64_t sbk,
                                              float *__restrict__ C, int64_t ldc, const float *__restrict__ bias,
                                              float *__restrict__ Z, int64_t ldz) {
  constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;  // LDS row pitch in bf16 (pads banks)
  __shared__ uint16_t As[TM * LDK];
  __shared__ uint16_t Bs[TN * LDK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TN;
  f16 acc = {};
  const bool a_kfast = sak == 1, b_kfast = sbk == 1;
  for (int k0 = 0; k0 < Kd; k0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += 256) {
      int mm, kk;
      if (a_kfast) {
        mm = e / TK;
        kk = e % TK;
      } else {
        mm = e % TM;
        kk = e / TM;
      }
      const int64_t gm = m0 + mm;
      const int gk = k0 + kk;
      As[mm * LDK + kk] = (gm < M && gk < Kd) ? f2bf(A[gm * sam + (int64_t)gk * sak]) : 0;
    }
    for (int e = threadIdx.x; e < TN * TK; e += 256) {
      int nn, kk;
      if (b_kfast) {
        nn = e / TK;
        kk = e % TK;
      } else {
        nn = e % TN;
        kk = e / TN;
      }
      const int64_t gn = n0 + nn;
      const int gk = k0 + kk;
      Bs[nn * LDK + kk] = (gn < N && gk < Kd) ? f2bf(Bm[gn * sbn + (int64_t)gk * sbk]) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
      // lane (i, g): A[i][ks + 8g .. +8], B[j][ks + 8g .. +8]
      const int i = lane & 31, g = lane >> 5;
      const uint4 av = *reinterpret_cast<const uint4 *>(As + (wm * 32 + i) * LDK + ks + 8 * g);
      const uint4 bv = *reinterpret_cast<const uint4 *>(Bs + (wn * 32 + i) * LDK + ks + 8 * g);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                    acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int jc = lane & 31, hf = lane >> 5;
  const int64_t gn = n0 + wn * 32 + jc;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t gm = m0 + wm * 32 + 8 * (v / 4) + 4 * hf + (v % 4);
    if (gm >= M || gn >= N) continue;
    float x = acc[v];
    if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) x += bias[gn];
    if (EPI == EPI_BIAS_GELU) {
      Z[gm * ldz + gn] = x;
      x = gelu(x);
    }
    if (EPI == EPI_GELU_GRAD) x *= gelu_grad(Z[gm * ldz + gn]);
    C[gm * ldc + gn] = x;
  }
}

template <int EPI>
static open_status gemm(open_ctx *ctx, const char *name, int M, int N, int Kd, const float *A, int64_t sam,
                        int64_t sak, const float *Bm, int64_t sbn, int64_t sbk, float *C, int64_t ldc,
                        const float *bias = nullptr, float *Z = nullptr, int64_t ldz = 0) {
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  OPEN_LAUNCH(ctx, name, k_gemm<EPI>, grid, dim3(256), 0, M, N, Kd, A, sam, sak, Bm, sbn, sbk, C, ldc, bias, Z, ldz);
  return OPEN_OK;
}

// ---------------------------------------------------------------- loss, reductions, Adam
// d_out = 2 (out - target) / (B k); block partial sums of (out - target)^2 in float64
__global__ __launch_bounds__(256) void k_loss(int64_t B, int k, const float *__restrict__ out,
                                              const int64_t *__restrict__ rows, const float *__restrict__ target,
                                              float *__restrict__ dout, double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t total = B * k;
  const float scale = 2.0f / (float)total;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t b = e / k, o = e % k;
    const int64_t i = rows ? rows[b] : b;
    const float d = out[e] - target[i * k + o];
    dout[e] = scale * d;
    acc += (double)d * (double)d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const double *__restrict__ part, int nparts, int64_t total, double *__restrict__ loss_d,
                             float *__restrict__ loss_f) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    s /= (double)total;
    if (loss_d) loss_d[0] = s;
    if (loss_f) loss_f[0] = (float)s;
  }
}

// out[c] = sum_b D[b][c] for c < N (bias gradients), fixed order
__global__ void k_colsum(int64_t B, int N, const float *__restrict__ D, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  float s = 0.f;
  for (int64_t b = 0; b < B; ++b) s += D[b * N + c];
  out[c] = s;
}

// Batch CSR gather: cnt[b] = |O_rows[b]|, then entries copied behind an exclusive scan.
__global__ void k_batch_count(int64_t B, const int64_t *__restrict__ rows, const int64_t *__restrict__ ptr,
                              int64_t *__restrict__ bptr) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    const int64_t i = rows ? rows[b] : b;
    bptr[b + 1] = ptr[i + 1] - ptr[i];
  }
  if (b == 0) bptr[0] = 0;
}

__global__ __launch_bounds__(1024) void k_inclusive_scan_i64(int64_t *__restrict__ x, int64_t len) {
  // single block, in place, len <= a few hundred thousand
  __shared__ int64_t part[1024];
  const int64_t per = (len + 1023) / 1024;
  const int64_t b0 = threadIdx.x * per, b1 = b0 + per < len ? b0 + per : len;
  int64_t acc = 0;
  for (int64_t i = b0; i < b1; ++i) acc += x[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int64_t i = b0; i < b1; ++i) {
    run += x[i];
    x[i] = run;
  }
}

__global__ void k_batch_gather(int64_t B, const int64_t *__restrict__ rows, const int64_t *__restrict__ ptr,
                               const int32_t *__restrict__ col, const float *__restrict__ val,
                               const int64_t *__restrict__ bptr, int n, int32_t *__restrict__ bcol,
                               float *__restrict__ bval) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < B; b += nw) {
    const int64_t i = rows ? rows[b] : b;
    const int64_t s = ptr[i], c = ptr[i + 1] - s, d = bptr[b];
    for (int64_t t = lane; t < c; t += 64) {
      bcol[d + t] = col[s + t];  // out-of-range columns are dropped by the column view
      bval[d + t] = val[s + t];
    }
  }
}

// Sparse W1 gradient: for input feature j (value part j, mask part n + j),
//   g[h][j]     = sum_{b: j in O_b} dz1[b][h] r_bj,   g[h][n + j] = sum_{b: j in O_b} dz1[b][h]
// one wavefront per feature over the batch's column view, lanes own 4 hidden units each.
__global__ __launch_bounds__(256) void k_grad_w1(int n, const int64_t *__restrict__ cp, const int32_t *__restrict__ rb,
                                                 const float *__restrict__ rv, const float *__restrict__ dz1,
                                                 float *__restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n) return;
  f4 gr = {0.f, 0.f, 0.f, 0.f}, gm = {0.f, 0.f, 0.f, 0.f};
  for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
    const f4 d = *reinterpret_cast<const f4 *>(dz1 + (int64_t)rb[e] * 256 + 4 * lane);
    const float r = rv[e];
    gr += r * d;
    gm += d;
  }
  const int64_t twon = 2 * (int64_t)n;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    g[(int64_t)(4 * lane + q) * twon + j] = gr[q];
    g[(int64_t)(4 * lane + q) * twon + n + j] = gm[q];
  }
}

__global__ void k_adam(int64_t np, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
}

// fallback decision: used[i] = !(rho_i <= tau) (NaN falls back), nonempty rows only
__global__ void k_fallback_flag(int64_t m, const int64_t *__restrict__ ptr, const float *__restrict__ rho, float tau,
                                uint8_t *__restrict__ used) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    used[i] = (ptr[i + 1] > ptr[i]) && !(rho[i] <= tau);
}

__global__ void k_count_u8(int64_t m, const uint8_t *__restrict__ f, int64_t *__restrict__ out) {
  __shared__ int64_t red[256];
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) c += f[i];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- fused inference
// Surrogate fold-in of a tile of kIR rows per block iteration (persistent grid), the network
// and the fallback test in one kernel: sparse first layer (each wavefront 16 rows, lane l
// hidden units 4l..4l+3) -> GELU -> bfloat16 tile in LDS -> second layer on BF16 MFMA with
// this wavefront's 64 columns of W2 held in registers for the whole kernel -> GELU -> LDS
// (over the first tile) -> third layer on MFMA -> u to global and LDS -> observed-entry RMS
// residual against the setting factors (four lanes per row) -> fallback flag.  Every
// arithmetic step matches the batched forward (same products, same order, same roundings).
constexpr int kIR = 64;       // rows per tile
constexpr int kHP = 256 + 8;  // LDS pitch of an activation row (bf16)

template <int K>
__global__ __launch_bounds__(256, 2) void k_mlp_infer(int64_t m, const int64_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col, const float *__restrict__ val,
                                                      int n, const uint16_t *__restrict__ W1T,
                                                      const float *__restrict__ b1, const float *__restrict__ W2,
                                                      const float *__restrict__ b2, const float *__restrict__ W3,
                                                      const float *__restrict__ b3, const float *__restrict__ F,
                                                      float tau, float *__restrict__ U, float *__restrict__ rho,
                                                      uint8_t *__restrict__ flag) {
  constexpr int CB3 = (K + 31) / 32;  // 32-column blocks of the output layer
  __shared__ __attribute__((aligned(16))) uint16_t Hs[kIR * kHP];
  __shared__ float Us[kIR * K];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i32 = lane & 31, g = lane >> 5;
  // B operands of the second layer: W2[64w + 32cb + i32][16ks + 8g .. +8] as bfloat16
  uint4 w2r[2][16];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const float *src = W2 + (int64_t)(64 * w + 32 * cb + i32) * 256 + 16 * ks + 8 * g;
      uint32_t pk[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) pk[e] = (uint32_t)f2bf(src[2 * e]) | ((uint32_t)f2bf(src[2 * e + 1]) << 16);
      w2r[cb][ks] = uint4{pk[0], pk[1], pk[2], pk[3]};
    }
  const float b2c[2] = {b2[64 * w + i32], b2[64 * w + 32 + i32]};
  const int64_t ntiles = (m + kIR - 1) / kIR;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * kIR;
    // ---- first layer (sparse), GELU, bfloat16 into LDS.  A row's entries are fetched 64 at
    // a time, one per lane, then taken in order, eight weight gathers in flight at once.
    for (int q = 0; q < 16; ++q) {
      const int lr = 16 * w + q;
      const int64_t row = r0 + lr;
      f4 z = *reinterpret_cast<const f4 *>(b1 + 4 * lane);
      const int64_t t0 = row < m ? ptr[row] : 0, t1 = row < m ? ptr[row + 1] : 0;
      for (int64_t base = t0; base < t1; base += 64) {
        const int nb = (int)(t1 - base < 64 ? t1 - base : 64);
        const int jl = lane < nb ? col[base + lane] : -1;
        const float rl = lane < nb ? val[base + lane] : 0.f;
        for (int u0 = 0; u0 < nb; u0 += 8) {
          uint2 wa[8], wm[8];
          int jj[8];
          float rr[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int t = u0 + e < nb ? u0 + e : nb - 1;
            jj[e] = __builtin_amdgcn_readlane(jl, t);
            rr[e] = readlane_f32(rl, t);
            const int js = (jj[e] >= 0 && jj[e] < n) ? jj[e] : 0;
            wa[e] = *reinterpret_cast<const uint2 *>(W1T + (int64_t)js * 256 + 4 * lane);
            wm[e] = *reinterpret_cast<const uint2 *>(W1T + (int64_t)(n + js) * 256 + 4 * lane);
          }
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if (u0 + e < nb && jj[e] >= 0 && jj[e] < n) {  // wave-uniform
              const float r = rr[e];
              z[0] += __builtin_fmaf(r, bf2f((uint16_t)(wa[e].x & 0xffff)), bf2f((uint16_t)(wm[e].x & 0xffff)));
              z[1] += __builtin_fmaf(r, bf2f((uint16_t)(wa[e].x >> 16)), bf2f((uint16_t)(wm[e].x >> 16)));
              z[2] += __builtin_fmaf(r, bf2f((uint16_t)(wa[e].y & 0xffff)), bf2f((uint16_t)(wm[e].y & 0xffff)));
              z[3] += __builtin_fmaf(r, bf2f((uint16_t)(wa[e].y >> 16)), bf2f((uint16_t)(wm[e].y >> 16)));
            }
          }
        }
      }
      const uint32_t lo = (uint32_t)f2bf(gelu(z[0])) | ((uint32_t)f2bf(gelu(z[1])) << 16);
      const uint32_t hi = (uint32_t)f2bf(gelu(z[2])) | ((uint32_t)f2bf(gelu(z[3])) << 16);
      *reinterpret_cast<uint2 *>(Hs + lr * kHP + 4 * lane) = uint2{lo, hi};
    }
    __syncthreads();
    // ---- second layer: this wavefront's 64 output columns for all kIR rows
    f16 acc[2][2] = {};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const uint4 a = *reinterpret_cast<const uint4 *>(Hs + (32 * rb + i32) * kHP + 16 * ks + 8 * g);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                               __builtin_bit_cast(bf16x8, w2r[cb][ks]), acc[rb][cb],
                                                               0, 0, 0);
      }
    }
    __syncthreads();  // every wavefront has read the first layer's tile
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rr = 32 * rb + 8 * (v / 4) + 4 * g + (v % 4);
          Hs[rr * kHP + 64 * w + 32 * cb + i32] = f2bf(gelu(acc[rb][cb][v] + b2c[cb]));
        }
    __syncthreads();
    // ---- third layer: tiles (row block, 32 outputs) on the first 2 CB3 wavefronts
    if (w < 2 * CB3) {
      const int rb = w & 1, cb = w >> 1;
      const int oc = 32 * cb + i32;  // output column supplied / received by this lane
      f16 acc3 = {};
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const uint4 a = *reinterpret_cast<const uint4 *>(Hs + (32 * rb + i32) * kHP + 16 * ks + 8 * g);
        uint32_t pk[4] = {0, 0, 0, 0};
        if (oc < K) {
          const float *src = W3 + (int64_t)oc * 256 + 16 * ks + 8 * g;
#pragma unroll
          for (int e = 0; e < 4; ++e) pk[e] = (uint32_t)f2bf(src[2 * e]) | ((uint32_t)f2bf(src[2 * e + 1]) << 16);
        }
        acc3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                      __builtin_bit_cast(bf16x8, uint4{pk[0], pk[1], pk[2], pk[3]}),
                                                      acc3, 0, 0, 0);
      }
      if (oc < K) {
        const float bias = b3[oc];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rr = 32 * rb + 8 * (v / 4) + 4 * g + (v % 4);
          const float x = acc3[v] + bias;
          Us[rr * K + oc] = x;
          if (r0 + rr < m) U[(r0 + rr) * K + oc] = x;
        }
      }
    }
    __syncthreads();
    // ---- observed-entry RMS residual: four lanes per row, K/4 dimensions each
    {
      constexpr int KQ = K / 4;
      const int lr = 16 * w + (lane >> 2), pq = lane & 3;
      const int64_t row = r0 + lr;
      int64_t t0 = 0, t1 = 0;
      if (row < m) {
        t0 = ptr[row];
        t1 = ptr[row + 1];
      }
      const int cnt = (int)(t1 - t0);
      int cmax = cnt;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(cmax, off, 64);
        cmax = o > cmax ? o : cmax;
      }
      float ssq = 0.f;
      for (int t0b = 0; t0b < cmax; t0b += 4) {
        // four entries in flight: indices and values, then the factor rows, then the dots
        int jv[4];
        float rv[4];
        const float *fv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = t0b + e;
          const bool in = t < cnt;
          jv[e] = in ? col[t0 + t] : -1;
          rv[e] = in ? val[t0 + t] : 0.f;
          const bool ok = jv[e] >= 0 && jv[e] < n;
          fv[e] = F + (int64_t)(ok ? jv[e] : 0) * K + pq * KQ;
        }
        float fx[4][KQ];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int a = 0; a < KQ; ++a) fx[e][a] = fv[e][a];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float d = 0.f;
#pragma unroll
          for (int a = 0; a < KQ; ++a) d = __builtin_fmaf(Us[lr * K + pq * KQ + a], fx[e][a], d);
          d += __shfl_xor(d, 1, 64);
          d += __shfl_xor(d, 2, 64);
          const float er = rv[e] - d;
          if (jv[e] >= 0 && jv[e] < n) ssq = __builtin_fmaf(er, er, ssq);
        }
      }
      if (pq == 0 && row < m) {
        const float rh = cnt > 0 ? sqrtf(ssq / (float)cnt) : 0.f;
        rho[row] = rh;
        flag[row] = (cnt > 0) && !(rh <= tau);
      }
    }
    __syncthreads();  // the tile buffers are reused
  }
}

}  // namespace openk

// ---------------------------------------------------------------- handle
struct open_mlp {
  open_ctx *ctx = nullptr;
  int n = 0, k = 0, H = 0;
  int64_t np = 0;
  int64_t off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
  float *w = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;  // masters, gradient, Adam moments
  uint16_t *w1t = nullptr;                                         // bf16 W1 transposed (2n x H)
  int64_t step = 0;
  // activations for a batch of up to cap rows
  int64_t cap = 0;
  float *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *out = nullptr, *dout = nullptr;
  float *d2 = nullptr, *d1 = nullptr;
  int64_t *bptr = nullptr;
  int32_t *bcol = nullptr;
  float *bval = nullptr;
  int64_t bnnz_cap = 0;
  int64_t *ccp = nullptr;
  int32_t *crb = nullptr;
  float *crv = nullptr;
  double *part = nullptr, *loss = nullptr;
  // inference scratch
  int64_t icap = 0;
  float *rho = nullptr;
  uint8_t *flag = nullptr;
  int64_t *cnt = nullptr;
};

namespace openk {

constexpr int kMaxBatchRows = 16384;
constexpr int kLossBlocks = 256;

static void mlp_free_batch(open_mlp *p) {
  float *fs[] = {p->z1, p->h1, p->z2, p->h2, p->out, p->dout, p->d2, p->d1, p->bval, p->crv};
  for (float *f : fs) (void)hipFree(f);
  (void)hipFree(p->bptr);
  (void)hipFree(p->bcol);
  (void)hipFree(p->ccp);
  (void)hipFree(p->crb);
  p->z1 = p->h1 = p->z2 = p->h2 = p->out = p->dout = p->d2 = p->d1 = p->bval = p->crv = nullptr;
  p->bptr = p->ccp = nullptr;
  p->bcol = p->crb = nullptr;
  p->cap = 0;
  p->bnnz_cap = 0;
}

static open_status mlp_batch_buffers(open_mlp *p, int64_t B, int64_t bnnz) {
  open_ctx *ctx = p->ctx;
  if (B > p->cap) {
    OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    float *keep_bval = p->bval, *keep_crv = p->crv;
    int32_t *keep_bcol = p->bcol, *keep_crb = p->crb;
    int64_t keep_bnnz = p->bnnz_cap;
    p->bval = p->crv = nullptr;
    p->bcol = p->crb = nullptr;
    mlp_free_batch(p);
    p->bval = keep_bval;
    p->crv = keep_crv;
    p->bcol = keep_bcol;
    p->crb = keep_crb;
    p->bnnz_cap = keep_bnnz;
    const size_t a = sizeof(float) * (size_t)B * p->H, o = sizeof(float) * (size_t)B * p->k;
    if (hipMalloc(&p->z1, a) || hipMalloc(&p->h1, a) || hipMalloc(&p->z2, a) || hipMalloc(&p->h2, a) ||
        hipMalloc(&p->out, o) || hipMalloc(&p->dout, o) || hipMalloc(&p->d2, a) || hipMalloc(&p->d1, a) ||
        hipMalloc(&p->bptr, sizeof(int64_t) * (B + 1)) || hipMalloc(&p->ccp, sizeof(int64_t) * (p->n + 1))) {
      (void)hipGetLastError();
      mlp_free_batch(p);
      return fail(ctx, OPEN_E_NOMEM, "surrogate batch buffers");
    }
    p->cap = B;
  }
  if (bnnz > p->bnnz_cap) {
    OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(p->bcol);
    (void)hipFree(p->bval);
    (void)hipFree(p->crb);
    (void)hipFree(p->crv);
    p->bcol = p->crb = nullptr;
    p->bval = p->crv = nullptr;
    const int64_t want = bnnz + bnnz / 4 + 64;
    if (hipMalloc(&p->bcol, sizeof(int32_t) * want) || hipMalloc(&p->bval, sizeof(float) * want) ||
        hipMalloc(&p->crb, sizeof(int32_t) * want) || hipMalloc(&p->crv, sizeof(float) * want)) {
      (void)hipGetLastError();
      return fail(ctx, OPEN_E_NOMEM, "surrogate batch buffers");
    }
    p->bnnz_cap = want;
  }
  return OPEN_OK;
}

static open_status mlp_repack(open_mlp *p) {
  OPEN_LAUNCH(p->ctx, "mlp_pack_w1t", k_pack_w1t, dim3(1024), dim3(256), 0, p->w, p->H, 2 * p->n, p->w1t);
  return OPEN_OK;
}

// forward over B rows (rows nullable) into p->out; saves z1, h1, z2, h2
static open_status mlp_forward_batch(open_mlp *p, int64_t B, const int64_t *rows, const int64_t *ptr,
                                     const int32_t *col, const float *val, float *out) {
  open_ctx *ctx = p->ctx;
  const int H = p->H, k = p->k;
  int64_t blocks = (B + 3) / 4;
  if (blocks > ctx->num_cu * 8) blocks = ctx->num_cu * 8;
  OPEN_LAUNCH(ctx, "mlp_layer1", k_layer1, dim3((unsigned)blocks), dim3(256), 0, B, rows, ptr, col, val, p->n, p->w1t,
              p->w + p->off_b1, p->z1, p->h1);
  open_status st;
  if ((st = gemm<EPI_BIAS_GELU>(ctx, "mlp_gemm_l2", (int)B, H, H, p->h1, H, 1, p->w + p->off_w2, H, 1, p->h2, H,
                                p->w + p->off_b2, p->z2, H)))
    return st;
  return gemm<EPI_BIAS>(ctx, "mlp_gemm_l3", (int)B, k, H, p->h2, H, 1, p->w + p->off_w3, H, 1, out, k,
                        p->w + p->off_b3);
}

// loss + gradient of the batch into p->g (and the loss scalar into loss_d / loss_f)
static open_status mlp_backward_batch(open_mlp *p, int64_t B, const int64_t *rows, const int64_t *ptr,
                                      const int32_t *col, const float *val, const float *target, double *loss_d,
                                      float *loss_f, int64_t bnnz_host) {
  open_ctx *ctx = p->ctx;
  const int H = p->H, k = p->k, n = p->n;
  open_status st;
  OPEN_LAUNCH(ctx, "mlp_loss", k_loss, dim3(kLossBlocks), dim3(256), 0, B, k, p->out, rows, target, p->dout, p->part);
  OPEN_LAUNCH(ctx, "mlp_loss_final", k_loss_final, dim3(1), dim3(64), 0, p->part, kLossBlocks, B * k, loss_d, loss_f);
  float *g = p->g;
  // layer 3: gW3[o][i] = sum_b dout[b][o] h2[b][i]; gb3 = sum_b dout
  if ((st = gemm<EPI_STORE>(ctx, "mlp_gemm_gw3", k, H, (int)B, p->dout, 1, k, p->h2, 1, H, g + p->off_w3, H))) return st;
  OPEN_LAUNCH(ctx, "mlp_colsum", k_colsum, dim3((k + 255) / 256), dim3(256), 0, B, k, p->dout, g + p->off_b3);
  // d2 = (dout W3) * GELU'(z2)
  if ((st = gemm<EPI_GELU_GRAD>(ctx, "mlp_gemm_dh2", (int)B, H, k, p->dout, k, 1, p->w + p->off_w3, 1, H, p->d2, H,
                                nullptr, p->z2, H)))
    return st;
  // layer 2: gW2[o][i] = sum_b d2[b][o] h1[b][i]; gb2
  if ((st = gemm<EPI_STORE>(ctx, "mlp_gemm_gw2", H, H, (int)B, p->d2, 1, H, p->h1, 1, H, g + p->off_w2, H))) return st;
  OPEN_LAUNCH(ctx, "mlp_colsum", k_colsum, dim3((H + 255) / 256), dim3(256), 0, B, H, p->d2, g + p->off_b2);
  // d1 = (d2 W2) * GELU'(z1)
  if ((st = gemm<EPI_GELU_GRAD>(ctx, "mlp_gemm_dh1", (int)B, H, H, p->d2, H, 1, p->w + p->off_w2, 1, H, p->d1, H,
                                nullptr, p->z1, H)))
    return st;
  OPEN_LAUNCH(ctx, "mlp_colsum", k_colsum, dim3((H + 255) / 256), dim3(256), 0, B, H, p->d1, g + p->off_b1);
  // sparse layer 1 over the batch's column view
  OPEN_LAUNCH(ctx, "mlp_batch_count", k_batch_count, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, B, rows, ptr,
              p->bptr);
  OPEN_LAUNCH(ctx, "mlp_batch_scan", k_inclusive_scan_i64, dim3(1), dim3(1024), 0, p->bptr + 1, B);
  OPEN_LAUNCH(ctx, "mlp_batch_gather", k_batch_gather, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, B, rows, ptr, col,
              val, p->bptr, n, p->bcol, p->bval);
  (void)bnnz_host;
  if ((st = csr_to_csc_dev(ctx, B, n, p->bptr, p->bcol, p->bval, p->ccp, p->crb, p->crv))) return st;
  OPEN_LAUNCH(ctx, "mlp_grad_w1", k_grad_w1, dim3((n + 3) / 4), dim3(256), 0, n, p->ccp, p->crb, p->crv, p->d1, g);
  return OPEN_OK;
}

static open_status batch_nnz(open_mlp *p, int64_t B, const int64_t *rows, const int64_t *ptr, int64_t *out) {
  // total observed entries of the batch rows, on the host (sizes the gather buffers)
  open_ctx *ctx = p->ctx;
  open_status st;
  if ((st = mlp_batch_buffers(p, B, 0))) return st;
  OPEN_LAUNCH(ctx, "mlp_batch_count", k_batch_count, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, B, rows, ptr,
              p->bptr);
  OPEN_LAUNCH(ctx, "mlp_batch_scan", k_inclusive_scan_i64, dim3(1), dim3(1024), 0, p->bptr + 1, B);
  int64_t *h;
  if ((st = pinned_get(ctx, 64, (void **)&h))) return st;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, p->bptr + B, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *out = h[0];
  return OPEN_OK;
}

}  // namespace openk

using namespace openk;

extern "C" {

int64_t open_mlp_num_params(int32_t n, int32_t k, int32_t hidden) {
  return (int64_t)hidden * 2 * n + hidden + (int64_t)hidden * hidden + hidden + (int64_t)k * hidden + k;
}

open_status open_mlp_create(open_ctx *ctx, open_mlp **out, int32_t n, int32_t k, int32_t hidden,
                            const float *init_host) {
  if (!ctx) return OPEN_E_INVALID;
  if (!out) return fail(ctx, OPEN_E_INVALID, "null output handle");
  *out = nullptr;
  if (hidden != 256) return fail(ctx, OPEN_E_UNSUPPORTED, "hidden width must be 256");
  if (!(k == 8 || k == 16 || k == 32 || k == 64)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (n <= 0 || n > 4096) return fail(ctx, OPEN_E_INVALID, "n must be in [1, 4096]");
  if (!init_host) return fail(ctx, OPEN_E_INVALID, "initial weights are required");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  open_mlp *p = new (std::nothrow) open_mlp();
  if (!p) return fail(ctx, OPEN_E_NOMEM, "handle");
  p->ctx = ctx;
  p->n = n;
  p->k = k;
  p->H = hidden;
  p->np = open_mlp_num_params(n, k, hidden);
  p->off_b1 = (int64_t)hidden * 2 * n;
  p->off_w2 = p->off_b1 + hidden;
  p->off_b2 = p->off_w2 + (int64_t)hidden * hidden;
  p->off_w3 = p->off_b2 + hidden;
  p->off_b3 = p->off_w3 + (int64_t)k * hidden;
  const size_t bytes = sizeof(float) * (size_t)p->np;
  if (hipMalloc(&p->w, bytes) || hipMalloc(&p->g, bytes) || hipMalloc(&p->am, bytes) || hipMalloc(&p->av, bytes) ||
      hipMalloc(&p->w1t, sizeof(uint16_t) * (size_t)hidden * 2 * n) ||
      hipMalloc(&p->part, sizeof(double) * (kLossBlocks + 8)) || hipMalloc(&p->loss, sizeof(double) * 8)) {
    (void)hipGetLastError();
    open_mlp_destroy(p);
    return fail(ctx, OPEN_E_NOMEM, "surrogate parameters");
  }
  open_status st = open_mlp_set_weights(p, init_host);
  if (st) {
    open_mlp_destroy(p);
    return st;
  }
  *out = p;
  return OPEN_OK;
}

open_status open_mlp_destroy(open_mlp *p) {
  if (!p) return OPEN_E_INVALID;
  if (p->ctx) (void)hipStreamSynchronize(p->ctx->stream);
  mlp_free_batch(p);
  (void)hipFree(p->w);
  (void)hipFree(p->g);
  (void)hipFree(p->am);
  (void)hipFree(p->av);
  (void)hipFree(p->w1t);
  (void)hipFree(p->part);
  (void)hipFree(p->loss);
  (void)hipFree(p->rho);
  (void)hipFree(p->flag);
  (void)hipFree(p->cnt);
  delete p;
  return OPEN_OK;
}

open_status open_mlp_get_weights(open_mlp *p, float *host_out) {
  if (!p || !host_out) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(host_out, p->w, sizeof(float) * p->np, hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return OPEN_OK;
}

open_status open_mlp_set_weights(open_mlp *p, const float *host_in) {
  if (!p || !host_in) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(p->w, host_in, sizeof(float) * p->np, hipMemcpyHostToDevice, ctx->stream));
  OPEN_LAUNCH(ctx, "fill", k_fill_i32, dim3(256), dim3(256), 0, (int *)p->am, p->np, 0);
  OPEN_LAUNCH(ctx, "fill", k_fill_i32, dim3(256), dim3(256), 0, (int *)p->av, p->np, 0);
  p->step = 0;
  open_status st = mlp_repack(p);
  if (st) return st;
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return OPEN_OK;
}

open_status open_mlp_forward(open_mlp *p, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *val,
                             float *U_hat) {
  if (!p) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  if (m < 0 || m >= INT32_MAX || (m > 0 && (!row_ptr || !col || !val || !U_hat)))
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  open_status st;
  for (int64_t b0 = 0; b0 < m; b0 += kMaxBatchRows) {
    const int64_t B = m - b0 < kMaxBatchRows ? m - b0 : kMaxBatchRows;
    if ((st = mlp_batch_buffers(p, B, 0))) return st;
    if ((st = mlp_forward_batch(p, B, nullptr, row_ptr + b0, col, val, U_hat + b0 * p->k))) return st;
  }
  return OPEN_OK;
}

open_status open_mlp_loss_grad(open_mlp *p, int64_t m, const int64_t *row_ptr, const int32_t *col,
                               const float *val, const float *target, double *loss, float *grads_host) {
  if (!p) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  if (m <= 0 || m > kMaxBatchRows || !row_ptr || !col || !val || !target || !loss || !grads_host)
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer (batch of 1..16384 rows)");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  open_status st;
  int64_t bnnz;
  if ((st = batch_nnz(p, m, nullptr, row_ptr, &bnnz))) return st;
  if ((st = mlp_batch_buffers(p, m, bnnz))) return st;
  if ((st = mlp_forward_batch(p, m, nullptr, row_ptr, col, val, p->out))) return st;
  if ((st = mlp_backward_batch(p, m, nullptr, row_ptr, col, val, target, p->loss, nullptr, bnnz))) return st;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(grads_host, p->g, sizeof(float) * p->np, hipMemcpyDeviceToHost, ctx->stream));
  double *h;
  if ((st = pinned_get(ctx, 64, (void **)&h))) return st;
  OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, p->loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  *loss = h[0];
  return OPEN_OK;
}

open_status open_mlp_train_step(open_mlp *p, int64_t m, const int64_t *row_ptr, const int32_t *col,
                                const float *val, const float *target, const int64_t *rows, int32_t batch, float lr,
                                float *loss_out) {
  if (!p) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  if (m <= 0 || m >= INT32_MAX || batch <= 0 || batch > kMaxBatchRows || (!rows && batch > m) || !row_ptr || !col ||
      !val || !target)
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer (batch of 1..16384 rows)");
  if (!(lr > 0.0f) || !isfinite(lr)) return fail(ctx, OPEN_E_INVALID, "learning rate must be finite and > 0");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  open_status st;
  // gather buffers sized for the longest possible batch: batch rows of at most n entries
  if ((st = mlp_batch_buffers(p, batch, (int64_t)batch * p->n))) return st;
  if ((st = mlp_forward_batch(p, batch, rows, row_ptr, col, val, p->out))) return st;
  if ((st = mlp_backward_batch(p, batch, rows, row_ptr, col, val, target, p->loss, loss_out, 0))) return st;
  p->step += 1;
  const float c1 = 1.0f - powf(0.9f, (float)p->step), c2 = 1.0f - powf(0.999f, (float)p->step);
  OPEN_LAUNCH(ctx, "mlp_adam", k_adam, dim3(1024), dim3(256), 0, p->np, p->w, p->g, p->am, p->av, lr, c1, c2);
  return mlp_repack(p);
}

open_status open_mlp_foldin(open_mlp *p, const float *F, int64_t m, const int64_t *row_ptr, const int32_t *col,
                            const float *val, float tau, float lambda, int32_t weighted, float *U_out,
                            uint8_t *used_fallback, float *rho, int64_t *n_fallback) {
  if (!p) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  if (m < 0 || m >= INT32_MAX || !F || (m > 0 && (!row_ptr || !col || !val || !U_out)))
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  if (!(tau >= 0.0f)) return fail(ctx, OPEN_E_INVALID, "tau must be >= 0");
  if (!(lambda >= 0.0f) || !isfinite(lambda)) return fail(ctx, OPEN_E_INVALID, "lambda must be finite and >= 0");
  if (m == 0) {
    if (n_fallback) *n_fallback = 0;
    return OPEN_OK;
  }
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  open_status st;
  if (m > p->icap) {
    OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    (void)hipFree(p->rho);
    (void)hipFree(p->flag);
    (void)hipFree(p->cnt);
    p->rho = nullptr;
    p->flag = nullptr;
    p->cnt = nullptr;
    if (hipMalloc(&p->rho, sizeof(float) * m) || hipMalloc(&p->flag, m) || hipMalloc(&p->cnt, sizeof(int64_t) * 512)) {
      (void)hipGetLastError();
      p->icap = 0;
      return fail(ctx, OPEN_E_NOMEM, "surrogate fold-in buffers");
    }
    p->icap = m;
  }
  float *r = rho ? rho : p->rho;
  uint8_t *f = used_fallback ? used_fallback : p->flag;
  // network, residual and fallback flag in one persistent kernel
  const int64_t tiles = (m + kIR - 1) / kIR;
  const unsigned grid = (unsigned)(tiles < (int64_t)ctx->num_cu * 2 ? tiles : (int64_t)ctx->num_cu * 2);
  const float *W = p->w;
  switch (p->k) {
    case 8:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<8>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1t,
                  W + p->off_b1, W + p->off_w2, W + p->off_b2, W + p->off_w3, W + p->off_b3, F, tau, U_out, r, f);
      break;
    case 16:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<16>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1t,
                  W + p->off_b1, W + p->off_w2, W + p->off_b2, W + p->off_w3, W + p->off_b3, F, tau, U_out, r, f);
      break;
    case 32:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<32>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1t,
                  W + p->off_b1, W + p->off_w2, W + p->off_b2, W + p->off_w3, W + p->off_b3, F, tau, U_out, r, f);
      break;
    default:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<64>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1t,
                  W + p->off_b1, W + p->off_w2, W + p->off_b2, W + p->off_w3, W + p->off_b3, F, tau, U_out, r, f);
      break;
  }
  // re-solve the flagged rows with the ridge fold-in (only they are bucketed)
  RowRef *list;
  int64_t *cls;
  if ((st = bucket_rows(ctx, m, row_ptr, p->k, &list, &cls, INT64_MAX, f))) return st;
  if ((st = rowsolve_launch(ctx, F, p->n, p->k, row_ptr, col, val, lambda, weighted, list, cls, U_out, nullptr, m)))
    return st;
  if (n_fallback) {
    OPEN_LAUNCH(ctx, "mlp_count_fallback", k_count_u8, dim3(256), dim3(256), 0, m, f, p->cnt);
    int64_t *h;
    if ((st = pinned_get(ctx, sizeof(int64_t) * 256, (void **)&h))) return st;
    OPEN_HIP_TRY(ctx, hipMemcpyAsync(h, p->cnt, sizeof(int64_t) * 256, hipMemcpyDeviceToHost, ctx->stream));
    OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    int64_t s = 0;
    for (int i = 0; i < 256; ++i) s += h[i];
    *n_fallback = s;
  }
  return OPEN_OK;
}

}  // extern "C"
