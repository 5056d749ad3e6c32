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
#include <limits.h>
#include <math.h>
#include <string.h>

#include <new>

#include "common.h"
#include "dense.h"

namespace openk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
// float32 -> bfloat16, round to nearest even (NaN stays NaN): the gfx950 conversion
// instruction v_cvt_pk_bf16_f32, two values at a time; bf16pack(a, b) has a in the low half
__device__ __forceinline__ uint32_t bf16pack(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf16x2v));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// GELU(z) = z Phi(z) (the erf form), with Phi(z) evaluated as the logistic function of an odd
// polynomial, Phi(z) ~ 1 / (1 + exp(-(a z + b z^3 + c z^5))), whose three coefficients were
// fitted to minimise the largest error of GELU over the real line (a = 1.5950157,
// b = 0.07401132, c = -7.030379e-4; the polynomial is taken at z clamped to [-10, 10], where
// it is increasing; GELU is taken as 0 below -10).  Largest absolute error of GELU: 2.5e-5,
// below the bfloat16 rounding of the activations that follows.  One exponential, one
// reciprocal and eight other instructions.
// The constants below are -log2(e) times the coefficients (the exponential is exp2).
constexpr float kGeluC0 = -2.301121234893799f, kGeluC1 = -0.10677576065063477f, kGeluC2 = 0.0010142693063244224f;
__device__ __forceinline__ float gelu_t(float z) {
  const float zc = __builtin_amdgcn_fmed3f(z, -10.0f, 10.0f);
  const float z2 = zc * zc;
  return zc * __builtin_fmaf(z2, __builtin_fmaf(z2, kGeluC2, kGeluC1), kGeluC0);
}
__device__ __forceinline__ float gelu(float z) {
  const float v = z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(gelu_t(z)));
  return z < -10.0f ? 0.0f : v;  // below -10 the clamped polynomial would leave z 9e-13
}
// SELU (Klambauer et al. 2017) and its derivative (the right-hand value at 0 is not taken: z > 0)
constexpr float kSeluA = 1.6732632423543772f, kSeluL = 1.0507009873554805f;
__device__ __forceinline__ float selu(float z) { return z > 0.f ? kSeluL * z : kSeluL * kSeluA * (__expf(z) - 1.f); }
__device__ __forceinline__ float selu_grad(float z) { return z > 0.f ? kSeluL : kSeluL * kSeluA * __expf(z); }
// derivative of the GELU above: s + z s'(z), s = 1 / (1 + e), e = 2^t(z),
// s' = -s^2 e ln2 t'(z), t' = C0 + 3 C1 z^2 + 5 C2 z^4 (0 where z is clamped)
__device__ __forceinline__ float gelu_grad(float z) {
  const float e = __builtin_amdgcn_exp2f(gelu_t(z));
  const float sg = __builtin_amdgcn_rcpf(1.0f + e);
  const float z2 = z * z;
  const float tp = __builtin_fabsf(z) < 10.0f
                       ? __builtin_fmaf(z2, __builtin_fmaf(z2, 5.0f * kGeluC2, 3.0f * kGeluC1), kGeluC0)
                       : 0.0f;
  return sg - z * sg * sg * e * 0.69314718055994531f * tp;
}

// ---------------------------------------------------------------- bfloat16 weight copies
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// First-layer weights as one 32-bit pair per (setting j, hidden unit h): low half
// bf16(W1[h][j]) (the weight of the value r_j), high half bf16(W1[h][n + j]) (the weight of the
// mask bit).  A lane's four units of one setting are one 16-byte load.
__global__ void k_pack_w1p(const float *__restrict__ W1, int H, int n, uint32_t *__restrict__ W1P) {
  const int64_t total = (int64_t)H * n, twon = 2 * (int64_t)n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / H, h = e % H;
    W1P[e] = bf16pack(W1[h * twon + j], W1[h * twon + n + j]);
  }
}

// W2 as the B operands of the inference kernel's second layer: entry ((w*2 + cb)*16 + ks)*64 +
// lane (lane = 32 g + i) holds W2[64w + 32cb + i][16ks + 8g .. +8] as 8 bfloat16.
__global__ void k_pack_w2p(const float *__restrict__ W2, uint4 *__restrict__ W2P) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8192) return;
  const int lane = e & 63, ks = (e >> 6) & 15, cb = (e >> 10) & 1, w = e >> 11;
  const int i = lane & 31, g = lane >> 5;
  const float *src = W2 + (int64_t)(64 * w + 32 * cb + i) * 256 + 16 * ks + 8 * g;
  uint32_t pk[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) pk[q] = bf16pack(src[2 * q], src[2 * q + 1]);
  W2P[e] = uint4{pk[0], pk[1], pk[2], pk[3]};
}

// W3 (K x 256) as the B operands of the inference kernel's output layer: entry
// (cb*16 + ks)*64 + lane (lane = 32 g + i) holds W3[32cb + i][16ks + 8g .. +8] as 8 bfloat16,
// zero for output rows past K.
__global__ void k_pack_w3p(const float *__restrict__ W3, int K, uint4 *__restrict__ W3P) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int cbs = (K + 31) / 32;
  if (e >= cbs * 1024) return;
  const int lane = e & 63, ks = (e >> 6) & 15, cb = e >> 10;
  const int o = 32 * cb + (lane & 31), g = lane >> 5;
  uint32_t pk[4] = {0, 0, 0, 0};
  if (o < K) {
    const float *src = W3 + (int64_t)o * 256 + 16 * ks + 8 * g;
#pragma unroll
    for (int q = 0; q < 4; ++q) pk[q] = bf16pack(src[2 * q], src[2 * q + 1]);
  }
  W3P[e] = uint4{pk[0], pk[1], pk[2], pk[3]};
}

// The value r of an observed entry as the pair (bf16(r), 1) that multiplies a weight pair
// (value weight, mask weight): one dot product adds a r + c.  The value is rounded to bfloat16
// like the weights (relative error at most 2^-9).  An entry whose column is outside [0, n)
// takes the pair (0, 0): it adds nothing.
__device__ __forceinline__ uint32_t value_pair(float r, bool valid) {
  return valid ? (uint32_t)f2bf(r) | (0x3f80u << 16) : 0u;
}

// The lane's weight pairs of setting j (four units, 16 bytes) from the packed first layer
// through a buffer resource over n settings: j outside [0, n) reads zeros.
__device__ __forceinline__ uint4 w1_pairs(__amdgpu_buffer_rsrc_t rs, int j, int lane) {
  const uint32_t off = ((uint32_t)j << 10) + 16u * (uint32_t)lane;  // j = -1 wraps out of range
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
}

// z += a r + c for the lane's four units (w: their weight pairs), one bfloat16 dot product
// per unit with float32 accumulation.  Every first-layer evaluation (training and inference)
// takes exactly these steps in the row's entry order.
__device__ __forceinline__ void layer1_step(f4 &z, uint4 w, uint32_t p) {
  const bf16x2 y = __builtin_bit_cast(bf16x2, p);
  const uint32_t wq[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) z[q] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, wq[q]), y, z[q], false);
}

// ---------------------------------------------------------------- sparse first layer
// One wavefront per batch row, lane l owns hidden units 4l..4l+3 (H = 256).
// rows (nullable) maps batch index b -> CSR row.  Writes z1 (nullable) and h1 = GELU(z1).
__global__ __launch_bounds__(256) void k_layer1(int64_t B, const int64_t *__restrict__ rows,
                                                const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                const float *__restrict__ val, int n,
                                                const uint32_t *__restrict__ W1P, const float *__restrict__ b1,
                                                float *__restrict__ z1, float *__restrict__ h1) {
  const int lane = threadIdx.x & 63;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(W1P, (uint64_t)n * 1024);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < B; b += nw) {
    const int64_t i = rows ? rows[b] : b;
    f4 z = *reinterpret_cast<const f4 *>(b1 + 4 * lane);
    for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t) {
      const int j = col[t];
      const bool ok = j >= 0 && j < n;
      layer1_step(z, w1_pairs(rs, ok ? j : -1, lane), value_pair(val[t], ok));
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


// Operand staging of the BF16 MFMA products.  A 64-row tile of X(r, k) = X[r*sr + k*sk] is
// staged one strip of up to kStripK k values at a time: every thread first issues all of its
// loads (8 chunks of 32 k, 8 values each, zero outside R x Kd), then packs each group of 8
// consecutive k into one 16-byte LDS store (bfloat16, round to nearest even, k-fast rows of
// pitch kLdk).  Threads are laid out so that global reads are contiguous across lanes: four
// threads per row when k is the fast index, 64 rows per k-group when the row is.
constexpr int kStripK = 256;
constexpr int kLdk = kStripK + 8;  // LDS row pitch in bf16 (pads banks)

__device__ __forceinline__ void strip_load(float (&v)[8][8], const float *__restrict__ X, int64_t sr, int64_t sk,
                                           int64_t r0, int64_t R, int k0, int Kd, bool kfast) {
  const int t = threadIdx.x;
  const int row = kfast ? t >> 2 : t & 63, kg = kfast ? t & 3 : t >> 6;
  const int64_t gr = r0 + row;
  const bool rok = gr < R;
  const float *base = X + (rok ? gr : 0) * sr;
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gk = k0 + 32 * c + 8 * kg + e;
      v[c][e] = (rok && gk < Kd) ? base[(int64_t)gk * sk] : 0.f;
    }
}

__device__ __forceinline__ void strip_store(uint16_t *__restrict__ Xs, const float (&v)[8][8], bool kfast, int nch) {
  const int t = threadIdx.x;
  const int row = kfast ? t >> 2 : t & 63, kg = kfast ? t & 3 : t >> 6;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    if (c < nch) {
      uint32_t pk[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) pk[e] = bf16pack(v[c][2 * e], v[c][2 * e + 1]);
      *reinterpret_cast<uint4 *>(Xs + row * kLdk + 32 * c + 8 * kg) = uint4{pk[0], pk[1], pk[2], pk[3]};
    }
  }
}

// acc += As[wm*32 .., 0..klen) x Bs[wn*32 .., 0..klen)^T on v_mfma_f32_32x32x16_bf16; lane (i, g)
// supplies A[i][ks + 8g .. +8] and B[j][ks + 8g .. +8]
__device__ __forceinline__ void strip_mfma(f16 &acc, const uint16_t *__restrict__ As, const uint16_t *__restrict__ Bs,
                                           int wm, int wn, int klen) {
  const int lane = threadIdx.x & 63, i = lane & 31, g = lane >> 5;
  const uint16_t *pa = As + (wm * 32 + i) * kLdk + 8 * g, *pb = Bs + (wn * 32 + i) * kLdk + 8 * g;
  for (int ks = 0; ks < klen; ks += 16) {
    const uint4 av = *reinterpret_cast<const uint4 *>(pa + ks);
    const uint4 bv = *reinterpret_cast<const uint4 *>(pb + ks);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                  acc, 0, 0, 0);
  }
}

// C[m][n] = epilogue(sum_k A(m, k) B(n, k)), A(m, k) = A[m*sam + k*sak], B(n, k) = B[n*sbn + k*sbk];
// block tile 64 x 64, four wavefronts of 32 x 32.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int Kd, const float *__restrict__ A, int64_t sam,
                                              int64_t sak, const float *__restrict__ Bm, int64_t sbn, int64_t sbk,
                                              float *__restrict__ C, int64_t ldc, const float *__restrict__ bias,
                                              float *__restrict__ Z, int64_t ldz) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * kLdk];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  f16 acc = {};
  for (int k0 = 0; k0 < Kd; k0 += kStripK) {
    const int klen = Kd - k0 < kStripK ? Kd - k0 : kStripK;
    float va[8][8], vb[8][8];
    strip_load(va, A, sam, sak, m0, M, k0, Kd, sak == 1);
    strip_load(vb, Bm, sbn, sbk, n0, N, k0, Kd, sbk == 1);
    if (k0 > 0) __syncthreads();  // the previous strip's LDS reads are done
    strip_store(As, va, sak == 1, (klen + 31) / 32);
    strip_store(Bs, vb, sbk == 1, (klen + 31) / 32);
    __syncthreads();
    strip_mfma(acc, As, Bs, wm, wn, klen);
  }
  const int jc = lane & 31, hf = lane >> 5;
  const int64_t gn = n0 + wn * 32 + jc;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t gm = m0 + wm * 32 + 8 * (v / 4) + 4 * hf + (v % 4);
    if (gm >= M || gn >= N) continue;
    float x = acc[v];
    if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU || EPI == EPI_BIAS_SELU) x += bias[gn];
    if (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS_SELU) {
      Z[gm * ldz + gn] = x;
      x = EPI == EPI_BIAS_GELU ? gelu(x) : selu(x);
    }
    if (EPI == EPI_GELU_GRAD) x *= gelu_grad(Z[gm * ldz + gn]);
    if (EPI == EPI_SELU_GRAD) x *= selu_grad(Z[gm * ldz + gn]);
    C[gm * ldc + gn] = x;
  }
}

// Weight gradient of a dense layer over a batch, split over the batch: slice s = blockIdx.z
// of kc batch rows writes
//   part[s][m][n] = sum_{b in s} A[b][m] Bv[b][n]     (bfloat16 products, float32 accumulation)
//   part[s][M*N + m] = sum_{b in s} A[b][m]            (the bias gradient, float32)
// with A = the layer's output gradient (Bsz x M, row-major) and Bv = its input (Bsz x N).  The
// slices are added in order by k_reduce_slices, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_gemm_wgrad(int M, int N, int Bsz, int kc, const float *__restrict__ A,
                                                    const float *__restrict__ Bv, float *__restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * kLdk];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * kLdk];
  __shared__ float bred[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int s = blockIdx.z;
  const int b0 = s * kc, b1 = b0 + kc < Bsz ? b0 + kc : Bsz;
  const float *Ag = A + (int64_t)b0 * M, *Bg = Bv + (int64_t)b0 * N;
  const int kd = b1 - b0;
  float bsum = 0.f;  // thread (row t % 64, k-group t / 64): its staged values of A, in order
  f16 acc = {};
  for (int k0 = 0; k0 < kd; k0 += kStripK) {
    const int klen = kd - k0 < kStripK ? kd - k0 : kStripK;
    float va[8][8], vb[8][8];
    // rows are the fast index of both operands (also when M or N is 1)
    strip_load(va, Ag, 1, M, m0, M, k0, kd, false);
    strip_load(vb, Bg, 1, N, n0, N, k0, kd, false);
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) bsum += va[c][e];
    if (k0 > 0) __syncthreads();
    strip_store(As, va, false, (klen + 31) / 32);
    strip_store(Bs, vb, false, (klen + 31) / 32);
    __syncthreads();
    strip_mfma(acc, As, Bs, wm, wn, klen);
  }
  float *dst = part + (int64_t)s * ((int64_t)M * N + M);
  const int jc = lane & 31, hf = lane >> 5;
  const int64_t gn = n0 + wn * 32 + jc;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t gm = m0 + wm * 32 + 8 * (v / 4) + 4 * hf + (v % 4);
    if (gm < M && gn < N) dst[gm * N + gn] = acc[v];
  }
  if (blockIdx.x == 0) {
    bred[threadIdx.x >> 6][threadIdx.x & 63] = bsum;
    __syncthreads();
    if (threadIdx.x < 64 && m0 + threadIdx.x < M)
      dst[(int64_t)M * N + m0 + threadIdx.x] =
          ((bred[0][threadIdx.x] + bred[1][threadIdx.x]) + bred[2][threadIdx.x]) + bred[3][threadIdx.x];
  }
}

// out[i] = sum_{s = 0..S-1} part[s][i] in slice order (eight slices' loads in flight)
__global__ __launch_bounds__(256) void k_reduce_slices(int64_t total, int S, const float *__restrict__ part,
                                                       float *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    float acc = 0.f;
    int s = 0;
    for (; s + 8 <= S; s += 8) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = part[(int64_t)(s + e) * total + i];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc += x[e];
    }
    for (; s < S; ++s) acc += part[(int64_t)s * total + i];
    out[i] = acc;
  }
}

// Dense input rows of a batch, x_b = [r * mask ; mask] (Bsz x 2n float32), one wavefront per
// row: the row is assembled in LDS (zeros, then its observed entries), then written out whole.
// Entries with a column outside [0, n) are left out, as in the sparse first layer.
__global__ __launch_bounds__(64) void k_dense_x(int64_t Bsz, const int64_t *__restrict__ rows,
                                                const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                const float *__restrict__ val, int n, float *__restrict__ X) {
  extern __shared__ float xs[];
  const int lane = threadIdx.x;
  const int twon = 2 * n;
  for (int64_t b = blockIdx.x; b < Bsz; b += gridDim.x) {
    for (int c = lane; c < twon; c += 64) xs[c] = 0.f;
    __syncthreads();
    const int64_t i = rows ? rows[b] : b;
    for (int64_t t = ptr[i] + lane; t < ptr[i + 1]; t += 64) {
      const int j = col[t];
      if (j >= 0 && j < n) {
        xs[j] = val[t];
        xs[n + j] = 1.0f;
      }
    }
    __syncthreads();
    float *dst = X + b * twon;
    for (int c = lane; c < twon; c += 64) dst[c] = xs[c];
    __syncthreads();
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

// Optimizer state on the device, so that a recorded training step can be replayed as is:
// t = Adam steps taken, cursor = batch index within the epoch, c1/c2 = bias corrections of
// the next step, 1 - beta1^(t+1) and 1 - beta2^(t+1).

__device__ __forceinline__ void train_state_set(TrainState *st, int64_t t) {
  st->t = t;
  st->c1 = (float)(1.0 - pow(0.9, (double)(t + 1)));
  st->c2 = (float)(1.0 - pow(0.999, (double)(t + 1)));
}

__global__ void k_train_state_reset(TrainState *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    train_state_set(st, 0);
    st->cursor = 0;
  }
}

// end of a training step: one more Adam step, next batch
__global__ void k_step_end(TrainState *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    train_state_set(st, st->t + 1);
    st->cursor += 1;
  }
}

__global__ void k_loss_final(const double *__restrict__ part, int nparts, int64_t total, double *__restrict__ loss_d,
                             float *__restrict__ loss_f, const TrainState *__restrict__ st,
                             float *__restrict__ loss_steps) {
  // lane l adds partials l, l + 64, ... in order, then a fixed butterfly combines the lanes
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int i = lane; i < nparts; i += 64) s += part[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    s /= (double)total;
    if (loss_d) loss_d[0] = s;
    if (loss_f) loss_f[0] = (float)s;
    if (loss_steps) loss_steps[st->t] = (float)s;
  }
}

// ---- seeded shuffle of the training rows, on the device
// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014): a 64-bit mixing bijection.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// perm[i] for i < m: a four-round balanced Feistel network on 2h-bit integers (4^h >= m,
// round keys key_r = mix64(mix64(seed) + 4 epoch + r), round function mix64(R ^ key_r) masked to
// h bits) is a bijection of [0, 4^h); walking its cycle from i until the value falls below m
// restricts it to a bijection of [0, m) (every cycle through i returns to i, so the walk ends).
// Thread 0 also rewinds the batch cursor of the epoch.
__global__ __launch_bounds__(256) void k_shuffle(int64_t m, int h, uint64_t seed, int64_t epoch,
                                                 int64_t *__restrict__ perm, TrainState *__restrict__ st) {
  const uint64_t base = mix64(seed) + 4ull * (uint64_t)epoch;
  uint64_t key[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) key[r] = mix64(base + (uint64_t)r);
  const uint64_t mask = (1ull << h) - 1ull;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    uint64_t x = (uint64_t)i;
    do {
      uint64_t L = x >> h, R = x & mask;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t nl = R;
        R = L ^ (mix64(R ^ key[r]) & mask);
        L = nl;
      }
      x = (L << h) | R;
    } while (x >= (uint64_t)m);
    perm[i] = (int64_t)x;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->cursor = 0;
}

// the rows of the current batch: rows[t] = perm[cursor * batch + t]
__global__ __launch_bounds__(256) void k_rows_of_step(const int64_t *__restrict__ perm, int batch,
                                                      const TrainState *__restrict__ st, int64_t *__restrict__ rows) {
  const int64_t off = st->cursor * (int64_t)batch;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < batch; t += gridDim.x * 256) rows[t] = perm[off + t];
}

__global__ void k_adam(int64_t np, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, const TrainState *__restrict__ st) {
  const float c1 = st->c1, c2 = st->c2;
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
// and the fallback test in one kernel:
//   first layer  each wavefront owns 16 consecutive rows, lane l hidden units 4l..4l+3.  The
//                row pointers of the 16 rows come in one load, their entries (contiguous in
//                the CSR) are staged in LDS up to kCap at a time, and the entries are taken as
//                one stream across the rows: the weight pairs of the next eight entries load
//                while the current eight are added, and a row is closed (GELU, bfloat16 into
//                the LDS tile) when the stream passes its end.
//   second layer BF16 MFMA, this wavefront's 64 output columns, its W2 operands streamed from
//                the packed copy (L2-resident) four steps ahead -> GELU -> LDS
//   third layer  MFMA -> u to global and LDS
//   residual     observed-entry RMS residual against the setting factors (four lanes per row;
//                the entries from the staging area when they fit) -> fallback flag.
// Every arithmetic step matches the batched forward (same products, same order, same
// roundings).
constexpr int kIR = 64;       // rows per tile
constexpr int kHP = 256 + 8;  // LDS pitch of an activation row (bf16)
constexpr int kCap = 176;     // entries staged per wavefront (three blocks per CU up to rank 32)
static_assert(kCap % 8 == 0, "a staged chunk is padded to a multiple of eight entries");

template <int K>
__global__ __launch_bounds__(256, 3) void k_mlp_infer(int64_t m, const int64_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col, const float *__restrict__ val,
                                                      int n, const uint32_t *__restrict__ W1P,
                                                      const float *__restrict__ b1, const uint4 *__restrict__ W2P,
                                                      const float *__restrict__ b2, const uint4 *__restrict__ W3P,
                                                      const float *__restrict__ b3, const float *__restrict__ F,
                                                      float tau, float *__restrict__ U, float *__restrict__ rho,
                                                      uint8_t *__restrict__ flag) {
  constexpr int CB3 = (K + 31) / 32;  // 32-column blocks of the output layer
  constexpr int PF = 4;               // W2 steps loaded ahead
  __shared__ __attribute__((aligned(16))) uint16_t Hs[kIR * kHP];
  __shared__ float Us[kIR * K];
  // per wavefront: {column or -1, value pair, value bits, 0} of its rows' entries
  __shared__ uint4 Stg[4][kCap];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i32 = lane & 31;
  const float b2c[2] = {b2[64 * w + i32], b2[64 * w + 32 + i32]};
  const f4 b1v = *reinterpret_cast<const f4 *>(b1 + 4 * lane);
  const uint2 hb1 = uint2{bf16pack(gelu(b1v[0]), gelu(b1v[1])), bf16pack(gelu(b1v[2]), gelu(b1v[3]))};
  const uint4 *w2w = W2P + (int64_t)(2 * w) * 16 * 64 + lane;  // step (cb, ks) at w2w[(cb*16 + ks)*64]
  const __amdgpu_buffer_rsrc_t rs1 = make_rsrc(W1P, (uint64_t)n * 1024);
  uint4 *stg = Stg[w];
  const int64_t ntiles = (m + kIR - 1) / kIR;
  // The next tile's row pointers and the first staged chunk of its entries are loaded while
  // the current tile is in its later phases.  Lane q <= 16 holds P_q, the first entry of row
  // 16 w + q of the tile (rows past m are empty); lane l holds entries l + 64 i of the chunk.
  constexpr int PK = (kCap + 63) / 64;
  auto load_ptrs = [&](int64_t tile) -> int64_t {
    const int64_t prow = tile * kIR + 16 * w + (lane < 16 ? lane : 16);
    return tile < ntiles ? ptr[prow < m ? prow : m] : 0;
  };
  int pcol[PK];
  float pval[PK];
  auto load_chunk0 = [&](int64_t pvn) {
    const int64_t e0 = readlane_i64(pvn, 0);
    const int64_t nn = readlane_i64(pvn, 16) - e0;
#pragma unroll
    for (int i = 0; i < PK; ++i) {
      const int t = lane + 64 * i;
      pcol[i] = t < nn && t < kCap ? col[e0 + t] : -1;
      pval[i] = t < nn && t < kCap ? val[e0 + t] : 0.f;
    }
  };
  int64_t pv_next = load_ptrs(blockIdx.x);
  load_chunk0(pv_next);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * kIR;
    // ---- first layer (sparse), GELU, bfloat16 into LDS
    const int64_t pv = pv_next;
    const int64_t E0 = readlane_i64(pv, 0);
    const int nent = (int)(readlane_i64(pv, 16) - E0);  // the wavefront's entries, < 2^31
    int cur = 0;                                      // row of the wavefront being accumulated
    int nxt = (int)(readlane_i64(pv, 1) - E0);        // first entry (relative) after it
    f4 z = b1v;
    auto advance = [&]() {
      ++cur;
      nxt = cur < 16 ? (int)(readlane_i64(pv, cur + 1) - E0) : INT_MAX;
    };
    // closes row cur (GELU, bfloat16 into the tile), then stores every following empty row
    // ending at or before entry u: rows without entries are GELU(b1)
    auto close_rows = [&](int u) {
      *reinterpret_cast<uint2 *>(Hs + (16 * w + cur) * kHP + 4 * lane) =
          uint2{bf16pack(gelu(z[0]), gelu(z[1])), bf16pack(gelu(z[2]), gelu(z[3]))};
      z = b1v;
      advance();
      while (u >= nxt) {
        *reinterpret_cast<uint2 *>(Hs + (16 * w + cur) * kHP + 4 * lane) = hb1;
        advance();
      }
    };
    for (int cs = 0; cs < nent; cs += kCap) {
      const int clen = nent - cs < kCap ? nent - cs : kCap;
      const int cpad = (clen + 7) & ~7;  // the chunk padded with entries that add nothing
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the previous chunk's reads of the staging area are done
      if (cs == 0) {
#pragma unroll
        for (int i = 0; i < PK; ++i) {
          const int t = lane + 64 * i;
          if (t < cpad) {
            const int j = pcol[i];
            const float r = pval[i];
            const bool ok = t < clen && j >= 0 && j < n;
            stg[t] = t < clen ? uint4{(uint32_t)(ok ? j : -1), value_pair(r, ok), __builtin_bit_cast(uint32_t, r), 0u}
                              : uint4{0xffffffffu, 0u, 0u, 0u};
          }
        }
      } else {
        for (int t = lane; t < cpad; t += 64) {
          uint4 e = uint4{0xffffffffu, 0u, 0u, 0u};
          if (t < clen) {
            const int j = col[E0 + cs + t];
            const float r = val[E0 + cs + t];
            const bool ok = j >= 0 && j < n;
            e = uint4{(uint32_t)(ok ? j : -1), value_pair(r, ok), __builtin_bit_cast(uint32_t, r), 0u};
          }
          stg[t] = e;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // two register sets of eight entries' weight pairs: one loads while the other is added
      uint4 wa[8], wb[8];
      uint32_t qa[8], qb[8];
      // the loads are issued in entry order (scheduling barriers), so that each entry waits
      // only for its own weights and not for the younger loads of the other set
      auto fetch = [&](uint4 (&wv)[8], uint32_t (&q)[8], int u0) {
        uint4 st[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) st[e] = stg[u0 + e];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          q[e] = st[e].y;
          wv[e] = w1_pairs(rs1, (int)st[e].x, lane);
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      // a padding entry adds exact zeros; a row it closes has ended at or before it
      auto consume = [&](const uint4 (&wv)[8], const uint32_t (&q)[8], int u0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          // rows end at one entry in ~14: the close is laid out of line, so that the common
          // path falls through instead of taking a branch per entry
          if (__builtin_expect(cs + u0 + e >= nxt, 0)) close_rows(cs + u0 + e);
          layer1_step(z, wv[e], q[e]);
        }
      };
      // Every fetch is unconditional (past the chunk it reloads entries 0..7, which are not
      // taken): a conditional one would make the waits count as if the other set had not been
      // issued, and each entry would wait for the younger loads too.
      fetch(wa, qa, 0);
      for (int u0 = 0; u0 < cpad; u0 += 16) {
        fetch(wb, qb, u0 + 8 < cpad ? u0 + 8 : 0);
        consume(wa, qa, u0);
        if (u0 + 8 >= cpad) break;
        fetch(wa, qa, u0 + 16 < cpad ? u0 + 16 : 0);
        consume(wb, qb, u0 + 8);
      }
    }
    if (cur < 16) close_rows(INT_MAX - 1);
    pv_next = load_ptrs(tile + gridDim.x);
    // the lane index through an opaque copy: the per-lane addresses of the later phases are
    // formed here in each tile instead of being hoisted out of the tile loop (and spilled)
    int lane_o = lane;
    asm volatile("" : "+v"(lane_o));
    const int i32o = lane_o & 31, go = (lane_o >> 5) & 1;
    __syncthreads();
    // ---- second layer: this wavefront's 64 output columns for all kIR rows
    f16 acc[2][2] = {};
    {
      // an offset the compiler cannot see through, so that the W2 loads stay in the tile loop
      // instead of being hoisted into 128 live registers
      int opq = 0;
      asm volatile("" : "+v"(opq));
      const uint4 *w2t = w2w + opq;
      uint4 ring[PF][2];
#pragma unroll
      for (int ks = 0; ks < PF; ++ks)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) ring[ks][cb] = w2t[(cb * 16 + ks) * 64];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const uint4 bw0 = ring[ks % PF][0], bw1 = ring[ks % PF][1];
        if (ks + PF < 16) {
          ring[ks % PF][0] = w2t[(ks + PF) * 64];
          ring[ks % PF][1] = w2t[(16 + ks + PF) * 64];
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const uint4 a = *reinterpret_cast<const uint4 *>(Hs + (32 * rb + i32o) * kHP + 16 * ks + 8 * go);
          acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                              __builtin_bit_cast(bf16x8, bw0), acc[rb][0], 0, 0, 0);
          acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                              __builtin_bit_cast(bf16x8, bw1), acc[rb][1], 0, 0, 0);
        }
      }
    }
    load_chunk0(pv_next);
    __syncthreads();  // every wavefront has read the first layer's tile
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rr = 32 * rb + 8 * (v / 4) + 4 * go + (v % 4);
          Hs[rr * kHP + 64 * w + 32 * cb + i32o] = f2bf(gelu(acc[rb][cb][v] + b2c[cb]));
        }
    __syncthreads();
    // ---- third layer: tiles (row block, 32 outputs) on the first 2 CB3 wavefronts
    if (w < 2 * CB3) {
      const int rb = w & 1, cb = w >> 1;
      const int oc = 32 * cb + i32o;  // output column supplied / received by this lane
      f16 acc3 = {};
      int opq = 0;
      asm volatile("" : "+v"(opq));  // keeps the operand loads in the tile loop
      const uint4 *w3t = W3P + cb * 16 * 64 + lane + opq;
      uint4 bw[16];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) bw[ks] = w3t[ks * 64];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const uint4 a = *reinterpret_cast<const uint4 *>(Hs + (32 * rb + i32o) * kHP + 16 * ks + 8 * go);
        acc3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, bw[ks]),
                                                      acc3, 0, 0, 0);
      }
      if (oc < K) {
        const float bias = b3[oc];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rr = 32 * rb + 8 * (v / 4) + 4 * go + (v % 4);
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
      constexpr int RQ = K <= 32 ? 8 : 4;  // entries per row in flight
      const int lr = 16 * w + (lane_o >> 2), pq = lane_o & 3;
      const int64_t row = r0 + lr;
      // the row's entries [P_q, P_q+1) from the lanes that loaded them (empty past m)
      const int q = lane_o >> 2;
      const int64_t t0 = (int64_t)(((uint64_t)(uint32_t)__shfl((int)((uint64_t)pv >> 32), q, 64) << 32) |
                                   (uint32_t)__shfl((int)(uint32_t)pv, q, 64));
      const int64_t t1 = (int64_t)(((uint64_t)(uint32_t)__shfl((int)((uint64_t)pv >> 32), q + 1, 64) << 32) |
                                   (uint32_t)__shfl((int)(uint32_t)pv, q + 1, 64));
      const int cnt = (int)(t1 - t0);
      int cmax = cnt;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(cmax, off, 64);
        cmax = o > cmax ? o : cmax;
      }
      float ssq = 0.f;
      const bool staged = nent <= kCap;  // wave-uniform: this row's entries are in stg
      const int sofs = (int)(t0 - E0);
      for (int t0b = 0; t0b < cmax; t0b += RQ) {
        // RQ entries in flight: indices and values, then the factor rows, then the dots
        int jv[RQ];
        float rv[RQ];
        const float *fv[RQ];
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          const int t = t0b + e;
          const bool in = t < cnt;
          if (staged) {
            const uint4 st = stg[in ? sofs + t : 0];
            jv[e] = in ? (int)st.x : -1;
            rv[e] = in ? __builtin_bit_cast(float, st.z) : 0.f;
          } else {
            jv[e] = in ? col[t0 + t] : -1;
            rv[e] = in ? val[t0 + t] : 0.f;
          }
          const bool okj = jv[e] >= 0 && jv[e] < n;
          fv[e] = F + (int64_t)(okj ? jv[e] : 0) * K + pq * KQ;
        }
        float fx[RQ][KQ];
#pragma unroll
        for (int e = 0; e < RQ; ++e)
#pragma unroll
          for (int a = 0; a < KQ; ++a) fx[e][a] = fv[e][a];
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
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
  uint32_t *w1p = nullptr;                                         // W1 weight pairs, bfloat16 (n x H)
  uint4 *w2p = nullptr;                                            // W2 as inference MFMA operands
  uint4 *w3p = nullptr;                                            // W3 as inference MFMA operands
  openk::TrainState *tstate = nullptr;                             // device optimizer state
  // activations for a batch of up to cap rows
  int64_t cap = 0;
  float *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *out = nullptr, *dout = nullptr;
  float *d2 = nullptr, *d1 = nullptr;
  float *xd = nullptr;     // dense input rows of the batch (batch x 2n), for the W1 gradient
  float *wpart = nullptr;  // split-over-the-batch partials of the weight and bias gradients
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

// batch slices of the weight-gradient product of an M x N layer: about 1024 blocks over the
// 64 x 64 output tiles, each slice a multiple of 32 batch rows
static int wgrad_slices(int64_t B, int M, int N, int *kc) {
  const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
  int64_t S = (1024 + tiles - 1) / tiles;
  if (S > 256) S = 256;
  int64_t c = (B + S - 1) / S;
  c = (c + 31) / 32 * 32;
  *kc = (int)c;
  return (int)((B + c - 1) / c);
}

// partial floats of an M x N weight gradient for any batch of at most B rows (the slice count
// does not grow with B, but a smaller batch can take up to its target count)
static int64_t wgrad_part_floats(int64_t B, int M, int N) {
  const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
  int64_t S = (1024 + tiles - 1) / tiles;
  if (S > 256) S = 256;
  const int64_t smax = (B + 31) / 32;  // slices are at least 32 rows
  return (S < smax ? S : smax) * ((int64_t)M * N + M);
}

static void mlp_free_batch(open_mlp *p) {
  float *fs[] = {p->z1, p->h1, p->z2, p->h2, p->out, p->dout, p->d2, p->d1, p->xd, p->wpart};
  for (float *f : fs) (void)hipFree(f);
  p->z1 = p->h1 = p->z2 = p->h2 = p->out = p->dout = p->d2 = p->d1 = p->xd = p->wpart = nullptr;
  p->cap = 0;
}

static open_status mlp_batch_buffers(open_mlp *p, int64_t B) {
  open_ctx *ctx = p->ctx;
  if (B <= p->cap) return OPEN_OK;
  if (ctx->capturing) return fail(ctx, OPEN_E_UNSUPPORTED, "buffer growth during graph capture");
  OPEN_HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  mlp_free_batch(p);
  const size_t a = sizeof(float) * (size_t)B * p->H, o = sizeof(float) * (size_t)B * p->k;
  const size_t x = sizeof(float) * (size_t)B * 2 * p->n;
  int64_t wp = wgrad_part_floats(B, p->k, p->H);
  if (wgrad_part_floats(B, p->H, p->H) > wp) wp = wgrad_part_floats(B, p->H, p->H);
  if (wgrad_part_floats(B, p->H, 2 * p->n) > wp) wp = wgrad_part_floats(B, p->H, 2 * p->n);
  if (hipMalloc(&p->z1, a) || hipMalloc(&p->h1, a) || hipMalloc(&p->z2, a) || hipMalloc(&p->h2, a) ||
      hipMalloc(&p->out, o) || hipMalloc(&p->dout, o) || hipMalloc(&p->d2, a) || hipMalloc(&p->d1, a) ||
      hipMalloc(&p->xd, x) || hipMalloc(&p->wpart, sizeof(float) * (size_t)wp)) {
    (void)hipGetLastError();
    mlp_free_batch(p);
    return fail(ctx, OPEN_E_NOMEM, "surrogate batch buffers");
  }
  p->cap = B;
  return OPEN_OK;
}

static open_status mlp_repack(open_mlp *p) {
  OPEN_LAUNCH(p->ctx, "mlp_pack_w1p", k_pack_w1p, dim3(1024), dim3(256), 0, p->w, p->H, p->n, p->w1p);
  OPEN_LAUNCH(p->ctx, "mlp_pack_w2p", k_pack_w2p, dim3(32), dim3(256), 0, p->w + p->off_w2, p->w2p);
  OPEN_LAUNCH(p->ctx, "mlp_pack_w3p", k_pack_w3p, dim3(8), dim3(256), 0, p->w + p->off_w3, p->k, p->w3p);
  return OPEN_OK;
}

// forward over B rows (rows nullable) into p->out; saves z1, h1, z2, h2
static open_status mlp_forward_batch(open_mlp *p, int64_t B, const int64_t *rows, const int64_t *ptr,
                                     const int32_t *col, const float *val, float *out) {
  open_ctx *ctx = p->ctx;
  const int H = p->H, k = p->k;
  int64_t blocks = (B + 3) / 4;
  if (blocks > ctx->num_cu * 8) blocks = ctx->num_cu * 8;
  OPEN_LAUNCH(ctx, "mlp_layer1", k_layer1, dim3((unsigned)blocks), dim3(256), 0, B, rows, ptr, col, val, p->n, p->w1p,
              p->w + p->off_b1, p->z1, p->h1);
  open_status st;
  if ((st = gemm<EPI_BIAS_GELU>(ctx, "mlp_gemm_l2", (int)B, H, H, p->h1, H, 1, p->w + p->off_w2, H, 1, p->h2, H,
                                p->w + p->off_b2, p->z2, H)))
    return st;
  return gemm<EPI_BIAS>(ctx, "mlp_gemm_l3", (int)B, k, H, p->h2, H, 1, p->w + p->off_w3, H, 1, out, k,
                        p->w + p->off_b3);
}

// weight and bias gradient of a dense layer (M outputs, N inputs) into g_w (M*N weights
// followed by M biases), split over the batch and reduced in slice order
static open_status wgrad(open_mlp *p, const char *name, int M, int N, int64_t B, const float *dY, const float *X,
                         float *g_w) {
  open_ctx *ctx = p->ctx;
  int kc;
  const int S = wgrad_slices(B, M, N, &kc);
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)S);
  OPEN_LAUNCH(ctx, name, k_gemm_wgrad, grid, dim3(256), 0, M, N, (int)B, kc, dY, X, p->wpart);
  const int64_t tot = (int64_t)M * N + M;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  OPEN_LAUNCH(ctx, "mlp_reduce_slices", k_reduce_slices, dim3((unsigned)blocks), dim3(256), 0, tot, S, p->wpart, g_w);
  return OPEN_OK;
}

// loss + gradient of the batch into p->g (and the loss scalar into loss_d / loss_f / the
// per-step record)
static open_status mlp_backward_batch(open_mlp *p, int64_t B, const int64_t *rows, const int64_t *ptr,
                                      const int32_t *col, const float *val, const float *target, double *loss_d,
                                      float *loss_f, float *loss_steps) {
  open_ctx *ctx = p->ctx;
  const int H = p->H, k = p->k, n = p->n;
  open_status st;
  OPEN_LAUNCH(ctx, "mlp_loss", k_loss, dim3(kLossBlocks), dim3(256), 0, B, k, p->out, rows, target, p->dout, p->part);
  OPEN_LAUNCH(ctx, "mlp_loss_final", k_loss_final, dim3(1), dim3(64), 0, p->part, kLossBlocks, B * k, loss_d, loss_f,
              p->tstate, loss_steps);
  float *g = p->g;
  // layer 3: gW3[o][i] = sum_b dout[b][o] h2[b][i], gb3 = sum_b dout[b]
  if ((st = wgrad(p, "mlp_wgrad_l3", k, H, B, p->dout, p->h2, g + p->off_w3))) return st;
  // d2 = (dout W3) * GELU'(z2)
  if ((st = gemm<EPI_GELU_GRAD>(ctx, "mlp_gemm_dh2", (int)B, H, k, p->dout, k, 1, p->w + p->off_w3, 1, H, p->d2, H,
                                nullptr, p->z2, H)))
    return st;
  // layer 2: gW2[o][i] = sum_b d2[b][o] h1[b][i], gb2 = sum_b d2[b]
  if ((st = wgrad(p, "mlp_wgrad_l2", H, H, B, p->d2, p->h1, g + p->off_w2))) return st;
  // d1 = (d2 W2) * GELU'(z1)
  if ((st = gemm<EPI_GELU_GRAD>(ctx, "mlp_gemm_dh1", (int)B, H, H, p->d2, H, 1, p->w + p->off_w2, 1, H, p->d1, H,
                                nullptr, p->z1, H)))
    return st;
  // layer 1: gW1[o][c] = sum_b d1[b][o] x_b[c] over the dense input rows, gb1 = sum_b d1[b]
  // (W1 and b1 are adjacent in the packing)
  int64_t xb = B < (int64_t)ctx->num_cu * 8 ? B : (int64_t)ctx->num_cu * 8;
  OPEN_LAUNCH(ctx, "mlp_dense_x", k_dense_x, dim3((unsigned)xb), dim3(64), sizeof(float) * 2 * n, B, rows, ptr, col,
              val, n, p->xd);
  return wgrad(p, "mlp_wgrad_l1", H, 2 * n, B, p->d1, p->xd, g);
}

// one Adam step on a batch (rows nullable: the first B rows), then the step counter
static open_status mlp_step(open_mlp *p, int64_t B, const int64_t *rows, const int64_t *ptr, const int32_t *col,
                            const float *val, const float *target, float lr, float *loss_out, float *loss_steps) {
  open_ctx *ctx = p->ctx;
  open_status st;
  if ((st = mlp_forward_batch(p, B, rows, ptr, col, val, p->out))) return st;
  if ((st = mlp_backward_batch(p, B, rows, ptr, col, val, target, p->loss, loss_out, loss_steps))) return st;
  OPEN_LAUNCH(ctx, "mlp_adam", k_adam, dim3(1024), dim3(256), 0, p->np, p->w, p->g, p->am, p->av, lr, p->tstate);
  OPEN_LAUNCH(ctx, "mlp_step_end", k_step_end, dim3(1), dim3(64), 0, p->tstate);
  return mlp_repack(p);
}

// ---------------------------------------------------------------- shared dense-training entry
// points (declared in dense.h; the NCF training composes them)
open_status dense_gemm(open_ctx *ctx, const char *name, int epi, int M, int N, int Kd, const float *A, int64_t sam,
                       int64_t sak, const float *Bm, int64_t sbn, int64_t sbk, float *C, int64_t ldc, const float *bias,
                       float *Z, int64_t ldz) {
  switch (epi) {
    case EPI_STORE: return gemm<EPI_STORE>(ctx, name, M, N, Kd, A, sam, sak, Bm, sbn, sbk, C, ldc, bias, Z, ldz);
    case EPI_BIAS: return gemm<EPI_BIAS>(ctx, name, M, N, Kd, A, sam, sak, Bm, sbn, sbk, C, ldc, bias, Z, ldz);
    case EPI_BIAS_SELU:
      return gemm<EPI_BIAS_SELU>(ctx, name, M, N, Kd, A, sam, sak, Bm, sbn, sbk, C, ldc, bias, Z, ldz);
    case EPI_SELU_GRAD:
      return gemm<EPI_SELU_GRAD>(ctx, name, M, N, Kd, A, sam, sak, Bm, sbn, sbk, C, ldc, bias, Z, ldz);
    default: return fail(ctx, OPEN_E_INVALID, "unknown GEMM epilogue");
  }
}

int64_t dense_wgrad_part_floats(int64_t B, int M, int N) { return wgrad_part_floats(B, M, N); }

open_status dense_wgrad(open_ctx *ctx, const char *name, int M, int N, int64_t B, const float *dY, const float *X,
                        float *part, float *g_w) {
  int kc;
  const int S = wgrad_slices(B, M, N, &kc);
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)S);
  OPEN_LAUNCH(ctx, name, k_gemm_wgrad, grid, dim3(256), 0, M, N, (int)B, kc, dY, X, part);
  const int64_t tot = (int64_t)M * N + M;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  OPEN_LAUNCH(ctx, "reduce_slices", k_reduce_slices, dim3((unsigned)blocks), dim3(256), 0, tot, S, part, g_w);
  return OPEN_OK;
}

open_status dense_train_state_reset(open_ctx *ctx, TrainState *st) {
  OPEN_LAUNCH(ctx, "train_state_reset", k_train_state_reset, dim3(1), dim3(64), 0, st);
  return OPEN_OK;
}

open_status dense_adam_step(open_ctx *ctx, int64_t np, float *w, const float *g, float *am, float *av, float lr,
                            TrainState *st) {
  OPEN_LAUNCH(ctx, "adam", k_adam, dim3(1024), dim3(256), 0, np, w, g, am, av, lr, st);
  OPEN_LAUNCH(ctx, "step_end", k_step_end, dim3(1), dim3(64), 0, st);
  return OPEN_OK;
}

open_status dense_loss_final(open_ctx *ctx, const double *part, int nparts, int64_t total, double *loss_d,
                             float *loss_f, const TrainState *st, float *loss_steps) {
  OPEN_LAUNCH(ctx, "loss_final", k_loss_final, dim3(1), dim3(64), 0, part, nparts, total, loss_d, loss_f, st,
              loss_steps);
  return OPEN_OK;
}

open_status dense_shuffle(open_ctx *ctx, int64_t m, uint64_t seed, int64_t epoch, int64_t *perm, TrainState *st) {
  int h = 1;
  while (h < 31 && (int64_t(1) << (2 * h)) < m) ++h;
  const int64_t blocks = (m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096;
  OPEN_LAUNCH(ctx, "shuffle", k_shuffle, dim3((unsigned)blocks), dim3(256), 0, m, h, seed, epoch, perm, st);
  return OPEN_OK;
}

open_status dense_rows_of_step(open_ctx *ctx, const int64_t *perm, int batch, const TrainState *st, int64_t *rows) {
  OPEN_LAUNCH(ctx, "rows_of_step", k_rows_of_step, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, perm, batch,
              st, rows);
  return OPEN_OK;
}

// Seeded initial weights: every weight and bias of a layer with fan-in f uniform on
// [-1/sqrt(f), 1/sqrt(f)), element e of the flat parameter vector drawn as
// (mix64(seed ^ mix64(e)) >> 40) * 2^-24 in [0, 1).
static void seeded_init(open_mlp *p, uint64_t seed, float *w) {
  struct Seg {
    int64_t off, len;
    int fan_in;
  };
  const int64_t H = p->H, n2 = 2 * (int64_t)p->n, k = p->k;
  const Seg seg[] = {{0, H * n2, (int)n2},          {p->off_b1, H, (int)n2}, {p->off_w2, H * H, (int)H},
                     {p->off_b2, H, (int)H},       {p->off_w3, k * H, (int)H}, {p->off_b3, k, (int)H}};
  for (const Seg &sg : seg) {
    const double a = 1.0 / sqrt((double)sg.fan_in);
    for (int64_t i = 0; i < sg.len; ++i) {
      const uint64_t e = (uint64_t)(sg.off + i);
      const double u = (double)(mix64(seed ^ mix64(e)) >> 40) * (1.0 / 16777216.0);
      w[sg.off + i] = (float)(a * (2.0 * u - 1.0));
    }
  }
}

}  // namespace openk

using namespace openk;

extern "C" {

int64_t open_mlp_num_params(int32_t n, int32_t k, int32_t hidden) {
  return (int64_t)hidden * 2 * n + hidden + (int64_t)hidden * hidden + hidden + (int64_t)k * hidden + k;
}

open_status open_mlp_create(open_ctx *ctx, open_mlp **out, int32_t n, int32_t k, int32_t hidden,
                            const float *init_host, uint64_t seed) {
  if (!ctx) return OPEN_E_INVALID;
  if (!out) return fail(ctx, OPEN_E_INVALID, "null output handle");
  *out = nullptr;
  if (hidden != 256) return fail(ctx, OPEN_E_UNSUPPORTED, "hidden width must be 256");
  if (!(k == 8 || k == 16 || k == 32 || k == 64)) return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  if (n <= 0 || n > 4096) return fail(ctx, OPEN_E_INVALID, "n must be in [1, 4096]");
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
      hipMalloc(&p->w1p, sizeof(uint32_t) * (size_t)hidden * n) || hipMalloc(&p->w2p, sizeof(uint4) * 8192) ||
      hipMalloc(&p->w3p, sizeof(uint4) * 2048) ||
      hipMalloc(&p->part, sizeof(double) * (kLossBlocks + 8)) || hipMalloc(&p->loss, sizeof(double) * 8) ||
      hipMalloc(&p->tstate, sizeof(TrainState))) {
    (void)hipGetLastError();
    open_mlp_destroy(p);
    return fail(ctx, OPEN_E_NOMEM, "surrogate parameters");
  }
  open_status st;
  if (init_host) {
    st = open_mlp_set_weights(p, init_host);
  } else {
    float *w0 = new (std::nothrow) float[(size_t)p->np];
    if (!w0) {
      open_mlp_destroy(p);
      return fail(ctx, OPEN_E_NOMEM, "initial weights");
    }
    seeded_init(p, seed, w0);
    st = open_mlp_set_weights(p, w0);
    delete[] w0;
  }
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
  (void)hipFree(p->w1p);
  (void)hipFree(p->w2p);
  (void)hipFree(p->w3p);
  (void)hipFree(p->tstate);
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
  OPEN_LAUNCH(ctx, "mlp_train_state_reset", k_train_state_reset, dim3(1), dim3(64), 0, p->tstate);
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
    if ((st = mlp_batch_buffers(p, B))) return st;
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
  if ((st = mlp_batch_buffers(p, m))) return st;
  if ((st = mlp_forward_batch(p, m, nullptr, row_ptr, col, val, p->out))) return st;
  if ((st = mlp_backward_batch(p, m, nullptr, row_ptr, col, val, target, p->loss, nullptr, nullptr))) return st;
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
  if ((st = mlp_batch_buffers(p, batch))) return st;
  return mlp_step(p, batch, rows, row_ptr, col, val, target, lr, loss_out, nullptr);
}

open_status open_mlp_train(open_mlp *p, int64_t m, const int64_t *row_ptr, const int32_t *col, const float *val,
                           const float *target, int32_t batch, float lr, int32_t epochs, uint64_t seed,
                           float *loss_hist) {
  if (!p) return OPEN_E_INVALID;
  open_ctx *ctx = p->ctx;
  if (m <= 0 || m >= INT32_MAX || !row_ptr || !col || !val || !target)
    return fail(ctx, OPEN_E_INVALID, "bad shape or pointer");
  if (batch <= 0 || batch > kMaxBatchRows || batch > m)
    return fail(ctx, OPEN_E_INVALID, "batch must be in [1, min(16384, m)]");
  if (epochs < 0) return fail(ctx, OPEN_E_INVALID, "epochs must be >= 0");
  if (!(lr > 0.0f) || !isfinite(lr)) return fail(ctx, OPEN_E_INVALID, "learning rate must be finite and > 0");
  if (epochs == 0) return OPEN_OK;
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int64_t spe = m / batch;  // full batches per epoch; the remainder is left to later shuffles
  const int64_t total = spe * epochs;
  int h = 1;
  while (h < 31 && (int64_t(1) << (2 * h)) < m) ++h;
  open_status st;
  if ((st = mlp_batch_buffers(p, batch))) return st;
  int64_t *perm = nullptr, *rows = nullptr;
  float *losses = nullptr;
  int64_t *t0h = nullptr;
  if (hipMalloc(&perm, sizeof(int64_t) * (size_t)m) || hipMalloc(&rows, sizeof(int64_t) * (size_t)batch) ||
      hipMalloc(&losses, sizeof(float) * (size_t)total)) {
    (void)hipGetLastError();
    (void)hipFree(perm);
    (void)hipFree(rows);
    (void)hipFree(losses);
    return fail(ctx, OPEN_E_NOMEM, "training buffers");
  }
  // the per-step losses are indexed by the Adam step count, which may not start at zero
  if ((st = pinned_get(ctx, 64, (void **)&t0h))) {
    (void)hipFree(perm);
    (void)hipFree(rows);
    (void)hipFree(losses);
    return st;
  }
  if (hipMemcpyAsync(t0h, p->tstate, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    (void)hipFree(perm);
    (void)hipFree(rows);
    (void)hipFree(losses);
    return fail(ctx, OPEN_E_DEVICE, "reading the step counter");
  }
  const int64_t t0 = t0h[0];
  float *loss_rec = losses - t0;  // loss of Adam step t lands in losses[t - t0]
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto one_step = [&]() -> open_status {
    OPEN_LAUNCH(ctx, "mlp_rows_of_step", k_rows_of_step, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, perm,
                batch, p->tstate, rows);
    return mlp_step(p, batch, rows, row_ptr, col, val, target, lr, nullptr, loss_rec);
  };
  const int64_t sblocks = (m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096;
  for (int32_t e = 0; e < epochs && st == OPEN_OK; ++e) {
    OPEN_LAUNCH(ctx, "mlp_shuffle", k_shuffle, dim3((unsigned)sblocks), dim3(256), 0, m, h, seed, (int64_t)e, perm,
                p->tstate);
    for (int64_t b = 0; b < spe && st == OPEN_OK; ++b) {
      if (!exec) {
        // the first step runs eagerly (it sizes every workspace), the next one is recorded
        if ((st = one_step())) break;
        if (b + 1 < spe || e + 1 < epochs) {
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
          for (int64_t b = 0; b < spe; ++b) sum += hl[e * spe + b];
          loss_hist[e] = (float)(sum / (double)spe);
        }
      }
      delete[] hl;
    }
  }
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(perm);
  (void)hipFree(rows);
  (void)hipFree(losses);
  return st;
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
  // resident blocks per CU: three (LDS about 50 KB each) up to rank 32, two at rank 64
  const int64_t per_cu = p->k == 64 ? 2 : 3;
  const unsigned grid = (unsigned)(tiles < (int64_t)ctx->num_cu * per_cu ? tiles : (int64_t)ctx->num_cu * per_cu);
  const float *W = p->w;
  switch (p->k) {
    case 8:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<8>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1p,
                  W + p->off_b1, p->w2p, W + p->off_b2, p->w3p, W + p->off_b3, F, tau, U_out, r, f);
      break;
    case 16:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<16>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1p,
                  W + p->off_b1, p->w2p, W + p->off_b2, p->w3p, W + p->off_b3, F, tau, U_out, r, f);
      break;
    case 32:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<32>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1p,
                  W + p->off_b1, p->w2p, W + p->off_b2, p->w3p, W + p->off_b3, F, tau, U_out, r, f);
      break;
    default:
      OPEN_LAUNCH(ctx, "mlp_infer", k_mlp_infer<64>, dim3(grid), dim3(256), 0, m, row_ptr, col, val, p->n, p->w1p,
                  W + p->off_b1, p->w2p, W + p->off_b2, p->w3p, W + p->off_b3, F, tau, U_out, r, f);
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
