// Batched ridge solves: fold-in of new rows and both ALS half-sweeps.
//
// For row i with observed set O_i (n_i entries), values r and fixed factors F (rows f_j):
//   primal  (n_i > k):  (F_O^T F_O + lambda w I_k) u = F_O^T r
//   dual    (n_i <= k): (F_O F_O^T + lambda w I_n) a = r,   u = F_O^T a
// (the same u by the push-through identity; w = n_i or 1).
//
// Layout: a wavefront solves 16 systems at once, four lanes per system ("quad").  A system
// of dimension D = 4N is stored as N x N tiles of 4x4; only tiles (I >= J) are kept.  Lane q
// of a quad holds, for every tile (I, J), column 4J+q of that tile (rows 4I..4I+3), which is
// exactly the output layout of v_mfma_f32_4x4x1_16b: block b of that instruction is quad b.
//   Gram    one 4x4x1 MFMA per tile and per contraction index (latent index for the dual
//           form, observation for the primal form); FP32 inputs, FP32 accumulation.
//   Solve   symmetric Gaussian elimination without pivoting (LDL^T, valid for SPD
//           matrices), the forward substitution fused into it, then column-oriented back
//           substitution.  Column p is broadcast inside the quad with DPP quad_perm.
//   Output  dual: u = F_O^T a, partial sums per lane, quad all-reduce with DPP;
//           primal: lane q holds u[4J+q] directly.
// Padded rows of a dual system (i >= n_i) have zero factors, unit diagonal and zero rhs,
// so their unknowns are exactly zero and do not touch the others.
#pragma once
#include "common.h"

namespace openk {

template <int N, int K, bool DUAL>
__device__ __forceinline__ void solve16(const float *__restrict__ F, int n, const int64_t *__restrict__ ptr,
                                        const int32_t *__restrict__ idx, const float *__restrict__ val, int64_t row,
                                        float lambda, int weighted, float *__restrict__ X,
                                        int32_t *__restrict__ status) {
  constexpr int T = N * (N + 1) / 2;
  constexpr int D = 4 * N;
  static_assert(DUAL || D == K, "primal systems are k x k");
  const int q = threadIdx.x & 3;
  int64_t beg = 0;
  int cnt = 0;
  if (row >= 0) {
    beg = ptr[row];
    cnt = (int)(ptr[row + 1] - beg);
  }
  f4 acc[T];
  sfor<0, T>([&](auto t) { acc[t] = f4{0.f, 0.f, 0.f, 0.f}; });
  float b[N];
  int nonfinite = 0, badidx = 0;
  int oi[DUAL ? N : 1];

  if constexpr (DUAL) {
    sfor<0, N>([&](auto J) {
      const int i = 4 * J + q;
      const bool ok = i < cnt;
      int j = ok ? idx[beg + i] : -1;
      if (ok && (j < 0 || j >= n)) {
        badidx = 1;
        j = -1;
      }
      oi[J] = j;
      const float r = ok ? val[beg + i] : 0.f;
      b[J] = r;
      nonfinite |= !__builtin_isfinite(r);
    });
    nonfinite |= quad_xor1_i(nonfinite);
    nonfinite |= quad_xor2_i(nonfinite);
    badidx |= quad_xor1_i(badidx);
    badidx |= quad_xor2_i(badidx);
    // Gram of the observed factor rows over the latent index
    for (int k0 = 0; k0 < K; k0 += 4) {
      f4 a[N];
      sfor<0, N>([&](auto J) {
        a[J] = oi[J] >= 0 ? *reinterpret_cast<const f4 *>(F + (int64_t)oi[J] * K + k0) : f4{0.f, 0.f, 0.f, 0.f};
      });
      sfor<0, 4>([&](auto kk) {
        sfor<0, N>([&](auto I) {
          sfor<0, I + 1>([&](auto J) {
            acc[tri(I, J)] = mfma4x4(a[I][(int)kk], a[J][(int)kk], acc[tri(I, J)]);
          });
        });
      });
    }
  } else {
    sfor<0, N>([&](auto J) { b[J] = 0.f; });
    // Gram of the observed factor rows over the observations (all 16 systems step together)
    const int tmax = wave_max_i(cnt);
    for (int t = 0; t < tmax; ++t) {
      bool ok = t < cnt;
      int j = ok ? idx[beg + t] : 0;
      if (ok && (j < 0 || j >= n)) {
        badidx = 1;
        ok = false;
      }
      const float r = ok ? val[beg + t] : 0.f;
      nonfinite |= !__builtin_isfinite(r);
      float a[N];
      sfor<0, N>([&](auto J) { a[J] = ok ? F[(int64_t)j * K + 4 * J + q] : 0.f; });
      sfor<0, N>([&](auto I) {
        sfor<0, I + 1>([&](auto J) { acc[tri(I, J)] = mfma4x4(a[I], a[J], acc[tri(I, J)]); });
      });
      sfor<0, N>([&](auto J) { b[J] = __builtin_fmaf(r, a[J], b[J]); });
    }
  }

  // ridge term on the diagonal (unit diagonal on padded rows of a dual system)
  const float reg = lambda * (weighted ? (float)cnt : 1.0f);
  sfor<0, N>([&](auto J) {
    const int c = 4 * J + q;
    const float dg = (!DUAL || c < cnt) ? reg : 1.0f;
    sfor<0, 4>([&](auto v) { acc[tri(J, J)][(int)v] += (q == (int)v) ? dg : 0.f; });
  });

  // elimination with fused forward substitution; column p is broadcast one row block at a time
  int bad = 0;
  sfor<0, D>([&](auto P) {
    constexpr int p = decltype(P)::value, Jp = p >> 2, qp = p & 3;
    const float d = quad_bcast_c<qp>(acc[tri(Jp, Jp)][qp]);
    bad |= !(d > 0.f);
    const float s = __builtin_amdgcn_rcpf(d);
    const float bp = quad_bcast_c<qp>(b[Jp]);
    float lc[N];
    sfor<Jp, N>([&](auto II) {
      constexpr int I = decltype(II)::value;
      float w[4];
      sfor<0, 4>([&](auto V) {
        constexpr int v = decltype(V)::value;
        if constexpr (4 * I + v > p)
          w[v] = quad_bcast_c<qp>(acc[tri(I, Jp)][v]);
        else
          w[v] = 0.f;
      });
      // multiplier of the lane's own column c = 4I+q:  G[c][p] / d  (0 for c <= p)
      lc[I] = (q == 0 ? w[0] : q == 1 ? w[1] : q == 2 ? w[2] : w[3]) * s;
      b[I] = __builtin_fmaf(-lc[I], bp, b[I]);
      sfor<Jp, I + 1>([&](auto JJ) {
        constexpr int Jc = decltype(JJ)::value;
        sfor<0, 4>([&](auto V) {
          constexpr int v = decltype(V)::value;
          if constexpr (4 * I + v > p) acc[tri(I, Jc)][v] = __builtin_fmaf(-w[v], lc[Jc], acc[tri(I, Jc)][v]);
        });
      });
    });
  });

  // back substitution
  float x[N], dotv[N];
  sfor<0, N>([&](auto J) {
    x[J] = 0.f;
    dotv[J] = 0.f;
  });
  sfor_down<0, D>([&](auto P) {
    constexpr int p = decltype(P)::value, Jp = p >> 2, qp = p & 3;
    const float d = quad_bcast_c<qp>(acc[tri(Jp, Jp)][qp]);
    const float xo = (b[Jp] - dotv[Jp]) * __builtin_amdgcn_rcpf(d);
    const float xp = quad_bcast_c<qp>(xo);
    x[Jp] = (q == qp) ? xp : x[Jp];
    sfor<0, Jp + 1>([&](auto Jc) { dotv[Jc] = __builtin_fmaf(acc[tri(Jp, Jc)][qp], xp, dotv[Jc]); });
  });

  const bool good = row >= 0 && cnt > 0 && !bad && !nonfinite && !badidx;
  if constexpr (DUAL) {
    // u = F_O^T a, four outputs at a time; lane q stores output k0 + q
    sfor<0, K / 4>([&](auto C) {
      constexpr int k0 = 4 * C;
      f4 uo = {0.f, 0.f, 0.f, 0.f};
      sfor<0, N>([&](auto J) {
        const f4 f = oi[J] >= 0 ? *reinterpret_cast<const f4 *>(F + (int64_t)oi[J] * K + k0) : f4{0.f, 0.f, 0.f, 0.f};
        sfor<0, 4>([&](auto e) { uo[(int)e] = __builtin_fmaf(x[J], f[(int)e], uo[(int)e]); });
      });
      sfor<0, 4>([&](auto e) {
        uo[(int)e] += quad_xor1(uo[(int)e]);
        uo[(int)e] += quad_xor2(uo[(int)e]);
      });
      if (row >= 0) {
        const float o = q == 0 ? uo[0] : q == 1 ? uo[1] : q == 2 ? uo[2] : uo[3];
        X[row * K + k0 + q] = good ? o : 0.f;
      }
    });
  } else {
    if (row >= 0) sfor<0, N>([&](auto J) { X[row * K + 4 * J + q] = good ? x[J] : 0.f; });
  }
  if (status && row >= 0 && q == 0)
    status[row] = cnt == 0      ? OPEN_ROW_EMPTY
                  : badidx    ? OPEN_ROW_BADINDEX
                  : nonfinite ? OPEN_ROW_NONFINITE
                  : bad       ? OPEN_ROW_NONPOS_PIVOT
                              : OPEN_ROW_OK;
}

template <int K, int N, int NHI>
__device__ __forceinline__ void dispatch_dual(int nmax, const float *F, int n, const int64_t *ptr, const int32_t *idx,
                                              const float *val, int64_t row, float lambda, int weighted, float *X,
                                              int32_t *status) {
  if constexpr (N < NHI) {
    if (nmax <= 4 * N) {
      solve16<N, K, true>(F, n, ptr, idx, val, row, lambda, weighted, X, status);
      return;
    }
    dispatch_dual<K, N + 1, NHI>(nmax, F, n, ptr, idx, val, row, lambda, weighted, X, status);
  } else {
    solve16<N, K, true>(F, n, ptr, idx, val, row, lambda, weighted, X, status);
  }
}

// Persistent kernel over the rows of classes c_lo..c_hi (contiguous in the bucketed list).
template <int K, int NLO, int NHI, bool DUAL>
__global__ __launch_bounds__(256) void k_solve_tier(const float *__restrict__ F, int n, const int64_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ idx, const float *__restrict__ val,
                                                    const int32_t *__restrict__ list, const int64_t *__restrict__ cls,
                                                    int c_lo, int c_hi, float lambda, int weighted,
                                                    float *__restrict__ X, int32_t *__restrict__ status) {
  const int64_t start = cls[2 * c_lo];
  const int64_t count = cls[2 * c_hi] + cls[2 * c_hi + 1] - start;
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); g * 16 < count; g += nw) {
    const int64_t slot = g * 16 + (lane >> 2);
    const int64_t row = slot < count ? (int64_t)list[start + slot] : -1;
    if constexpr (DUAL) {
      const int cnt = row >= 0 ? (int)(ptr[row + 1] - ptr[row]) : 0;
      const int nmax = wave_max_i(cnt);
      dispatch_dual<K, NLO, NHI>(nmax, F, n, ptr, idx, val, row, lambda, weighted, X, status);
    } else {
      solve16<K / 4, K, false>(F, n, ptr, idx, val, row, lambda, weighted, X, status);
    }
  }
}

// Launch one tier kernel (classes c_lo..c_hi) with a persistent grid sized for m rows.
template <int K, int NLO, int NHI, bool DUAL>
open_status launch_tier(const char *name, open_ctx *ctx, const float *F, int n, const int64_t *ptr, const int32_t *idx, const float *val,
                        float lambda, int weighted, const int32_t *list, const int64_t *cls, int c_lo, int c_hi,
                        float *X, int32_t *status, int64_t m) {
  const int64_t groups = (m + 15) / 16;
  int64_t blocks = (groups + 3) / 4;
  const int64_t cap = (int64_t)ctx->num_cu * 4;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  OPEN_LAUNCH(ctx, name, (k_solve_tier<K, NLO, NHI, DUAL>), dim3((unsigned)blocks), dim3(256), 0, F, n, ptr, idx, val,
              list, cls, c_lo, c_hi, lambda, weighted, X, status);
  return OPEN_OK;
}

#define OPEN_TIER_ARGS                                                                                       \
  open_ctx *ctx, const float *F, int n, const int64_t *ptr, const int32_t *idx, const float *val, float lambda, \
      int weighted, const int32_t *list, const int64_t *cls, float *X, int32_t *status, int64_t m
#define OPEN_TIER_PASS ctx, F, n, ptr, idx, val, lambda, weighted, list, cls
// one function per (rank, tier), each compiled in its own translation unit
open_status tier_k8_dual(OPEN_TIER_ARGS);
open_status tier_k8_primal(OPEN_TIER_ARGS);
open_status tier_k16_dual(OPEN_TIER_ARGS);
open_status tier_k16_primal(OPEN_TIER_ARGS);
open_status tier_k32_d14(OPEN_TIER_ARGS);
open_status tier_k32_d56(OPEN_TIER_ARGS);
open_status tier_k32_d78(OPEN_TIER_ARGS);
open_status tier_k32_primal(OPEN_TIER_ARGS);
open_status tier_k64_d14(OPEN_TIER_ARGS);
open_status tier_k64_d56(OPEN_TIER_ARGS);
open_status tier_k64_d78(OPEN_TIER_ARGS);

}  // namespace openk
