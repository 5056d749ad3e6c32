// Batched ridge solves: fold-in of new rows and both ALS half-sweeps.
//
// For row i with observed set O_i (n_i entries), values r and fixed factors F (rows f_j):
//   primal  (n_i > k):  (F_O^T F_O + lambda w I_k) u = F_O^T r
//   dual    (n_i <= k): (F_O F_O^T + lambda w I_n) a = r,   u = F_O^T a
// (the same u by the push-through identity; w = n_i or 1).
//
// One persistent kernel per size class.  A wavefront solves a group of 64/P systems of one
// class, P lanes per system (P = 1, 2 or 4), padded dimension D.
//
//   Stage  A persistent block copies the factor matrix F into LDS once when it fits (the
//          fold-in's 480 x 32 setting factors do); every factor-row gather then reads LDS.
//          Each lane fetches the column indices and values of its own system once per group
//          and shares them with the other lanes through LDS.
//   Gram   In sub-batches of 16 systems (quad b of the wave = system b of the sub-batch) the
//          system is kept as 4x4 tiles (lower block triangle only): one 4x4x1 MFMA
//          (v_mfma_f32_4x4x1_16b) per tile and contraction index - the latent index for the
//          dual form, the observation for the primal form.  FP32 inputs and accumulation.
//          The instruction's output puts column 4J+q of tile (I, J) in lane q of the quad.
//   Layout The P lanes of a system own its columns interleaved: lane pi owns c = P m + pi and
//          keeps rows P m .. D-1 of them in registers; for P < 4 the lower triangle passes
//          through a per-wave LDS buffer.  With P = 4 the lanes own rows instead (lane pi: row
//          4I + pi, columns 0 .. 4I + 3), which the MFMA writes directly when its operands are
//          swapped; the blocked elimination keeps the column layout.
//   Solve  Right-looking symmetric Gaussian elimination (LDL^T, no pivoting: the systems are
//          SPD) with the forward substitution fused in, then the back substitution (column-
//          oriented; with owned rows, a sum per lane and a quad reduction per unknown).  Pivot
//          columns move between the P lanes by DPP quad_perm; with P = 1 no data moves at all.
//   Output dual: each lane forms K/P outputs of u = F_O^T a from its system's factor rows;
//          primal: the solution is u itself.
// Padded rows of a dual system (i >= n_i) have zero factors, unit diagonal and zero rhs:
// their unknowns are exactly zero and they do not touch the others.
#pragma once
#include "common.h"

namespace openk {

// DPP broadcast of lane `src` of each group of P lanes (P = 1, 2, 4) inside the quad
template <int P, int SRC>
__device__ __forceinline__ float grp_bcast(float x) {
  if constexpr (P == 1) {
    return x;
  } else if constexpr (P == 2) {
    constexpr int c = SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), c, 0xf, 0xf, true));
  } else {
    return quad_bcast_c<SRC>(x);
  }
}

// v[pi] for the lane's position pi in its group (compile-time array, runtime pi), as
// selects on the bits of pi (a compare chain would become a branchy switch)
template <int P>
__device__ __forceinline__ float pick(const float *v, int pi) {
  if constexpr (P == 1) return v[0];
  const bool b0 = pi & 1;
  if constexpr (P == 2) return b0 ? v[1] : v[0];
  const float lo = b0 ? v[1] : v[0], hi = b0 ? v[3] : v[2];
  return (pi & 2) ? hi : lo;
}

// ---------------------------------------------------------------- factor-row access
// F rows from LDS or from global memory through a bounds-checked buffer resource.  In LDS a
// row occupies K + 4 floats (one pad chunk, so that lanes reading the same chunk of different
// rows spread over the banks) and a row of zeros sits just before row 0: the row index -1 of
// padded and rejected entries reads zeros without a test, as it does from the buffer
// resource (a negative offset is out of range there).
template <int K, bool LDS>
struct FRows {
  static constexpr int PS = K + 4;  // LDS row pitch in floats
  const float *lds;                 // row 0 (row -1 is the zero row)
  __amdgpu_buffer_rsrc_t rs;
  __device__ __forceinline__ f4 row4(int j, int k0) const {
    if constexpr (LDS)
      return *reinterpret_cast<const f4 *>(lds + j * PS + k0);
    else
      return bload_f4(rs, (j * K + k0) * 4);
  }
  __device__ __forceinline__ float row1(int j, int k) const {
    if constexpr (LDS)
      return lds[j * PS + k];
    else
      return bload_f32(rs, (j * K + k) * 4);
  }
};

// LDS per wave (floats): lower triangles of one sub-batch (P < 4), the group's column
// indices and values, and per-system bookkeeping
__host__ __device__ constexpr int tri_stride(int D) { return (D * (D + 1) / 2) | 1; }
__host__ __device__ constexpr int wave_lds_floats(int P, int D) {
  return (P < 4 ? 16 * tri_stride(D) : 0) + 2 * (64 / P) * (D + 1);
}

template <int P, int D, int K, bool DUAL, bool LDSF, bool PF, bool BLK>
__device__ __forceinline__ void solve_group(const FRows<K, LDSF> &Fr, int n, const RowRef mine,
                                            const int32_t *__restrict__ idx, const float *__restrict__ val,
                                            float lambda, int weighted, float *__restrict__ X,
                                            int32_t *__restrict__ status, float *__restrict__ wl) {
  constexpr int N = D / 4;            // tiles per dimension
  constexpr int T = N * (N + 1) / 2;  // lower block triangle
  constexpr int M = D / P;            // columns owned per lane
  constexpr int SB = 4 / P;           // sub-batches of 16 systems
  constexpr int SYS = 64 / P;         // systems per wave
  constexpr int ST = tri_stride(D);
  constexpr int E = D + 1;            // LDS pitch of a system's index/value lists
  static_assert(D % 4 == 0 && D % P == 0, "shape");
  static_assert(DUAL || D == K, "primal systems are k x k");
  // Four lanes per system (not blocked) own rows instead of columns: lane pi holds
  // st[I][j] = G[4I + pi][j], j = 0 .. 4I + 3, so that an elimination step's multipliers are the
  // lane's own entries and only the pivot column's entries travel between lanes.
  constexpr bool ROW = P == 4 && !BLK;
  const int lane = threadIdx.x & 63;
  const int pi = lane % P;  // position in the system's lane group
  const int qi = lane & 3;  // position in the quad (MFMA layout)
  const int sme = lane / P;  // this lane's system in the group
  float *tri_buf = wl;                                       // [16][ST]      (P < 4)
  int *ixs = reinterpret_cast<int *>(wl + (P < 4 ? 16 * ST : 0));  // [SYS][E] column indices (-1 = none)
  float *vxs = wl + (P < 4 ? 16 * ST : 0) + SYS * E;               // [SYS][E] values

  // ---- this lane's system (record prefetched by the caller): row, range, flags; its
  // index/value lists into LDS
  const int64_t my_row = mine.row;
  const int64_t mbeg = mine.beg;
  const int my_cnt = mine.cnt;
  int my_flags = 0;  // 1: non-finite value, 2: column index out of range
  if constexpr (DUAL) {
    // lane pi of the group fetches entries pi, pi + P, ...
    const bool any_obs = __any(my_cnt > 0);
    sfor<0, M>([&](auto Mm) {
      const int i = P * Mm + pi;
      const bool ok = i < my_cnt;
      const int64_t e = ok ? mbeg + i : 0;
      int j = -1;
      float r = 0.f;
      if (any_obs) {
        j = idx[e];
        r = val[e];
      }
      if (ok && (j < 0 || j >= n)) my_flags |= 2;
      if (ok && !__builtin_isfinite(r)) my_flags |= 1;
      ixs[sme * E + i] = (ok && j >= 0 && j < n) ? j : -1;
      vxs[sme * E + i] = ok ? r : 0.f;
    });
    if constexpr (P == 2) my_flags |= __builtin_amdgcn_mov_dpp(my_flags, 0xb1, 0xf, 0xf, true);
    if constexpr (P == 4) {
      my_flags |= quad_xor1_i(my_flags);
      my_flags |= quad_xor2_i(my_flags);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // owned columns: st[m][j] = G[P m + j][P m + pi], j = 0 .. D - P m - 1
  float st[M][D];
  float pb[DUAL ? 1 : N];  // primal rhs in the quad layout: pb[J] = (F_O^T r)[4J + qi]
  int pflags = 0;
  if constexpr (!DUAL) sfor<0, N>([&](auto J) { pb[J] = 0.f; });

#pragma unroll 1
  for (int sb = 0; sb < SB; ++sb) {
    // ---- quad b of the wave works on system qs = 16 sb + b (quad-layout view)
    const int qs = 16 * sb + (lane >> 2);
    const int qsrc = qs * P;  // a lane of that system (holds its count)
    const int cnt = __shfl(my_cnt, qsrc, 64);
    f4 acc[T];
    sfor<0, T>([&](auto t) { acc[t] = f4{0.f, 0.f, 0.f, 0.f}; });
    // the MFMA phase issues at raised priority, so a wave in its Gram keeps the matrix pipe
    // fed while the SIMD's other waves run their (VALU-bound) eliminations in the gaps
    __builtin_amdgcn_s_setprio(1);
    if constexpr (DUAL) {
      int oi[N];
      sfor<0, N>([&](auto J) { oi[J] = ixs[qs * E + 4 * J + qi]; });
      f4 a[N];
      sfor<0, N>([&](auto J) { a[J] = Fr.row4(oi[J], 0); });
      sfor<0, K / 4>([&](auto C) {
        constexpr int k0 = 4 * C;
        f4 an[N];  // with PF, the next chunk is read while this one feeds the MFMAs
        if constexpr (PF && k0 + 4 < K) sfor<0, N>([&](auto J) { an[J] = Fr.row4(oi[J], k0 + 4); });
        sfor<0, 4>([&](auto kk) {
          sfor<0, N>([&](auto I) {
            sfor<0, I + 1>([&](auto J) {
              // row-owned layout: the transposed tile (lane q: row 4I + q, register v: column 4J + v)
              if constexpr (ROW)
                acc[tri(I, J)] = mfma4x4(a[J][(int)kk], a[I][(int)kk], acc[tri(I, J)]);
              else
                acc[tri(I, J)] = mfma4x4(a[I][(int)kk], a[J][(int)kk], acc[tri(I, J)]);
            });
          });
        });
        if constexpr (k0 + 4 < K) {
          if constexpr (PF)
            sfor<0, N>([&](auto J) { a[J] = an[J]; });
          else
            sfor<0, N>([&](auto J) { a[J] = Fr.row4(oi[J], k0 + 4); });
        }
      });
    } else {
      // primal: contraction over the observations of the 16 systems, in step
      const int64_t qbeg = (int64_t)(uint32_t)__shfl((int)(mbeg & 0xffffffff), qsrc, 64) |
                           ((int64_t)__shfl((int)(mbeg >> 32), qsrc, 64) << 32);
      const int tmax = wave_max_i(cnt);
      // indices and values PD entries ahead of the contraction
      constexpr int PD = 4;
      int jn[PD];
      float rn[PD];
      auto fetch = [&](int t0) {
        sfor<0, PD>([&](auto E) {
          const int t = t0 + (int)E;
          const int64_t e = t < cnt ? qbeg + t : (cnt > 0 ? qbeg : 0);
          jn[E] = idx[e];
          rn[E] = val[e];
        });
      };
      if (tmax > 0) fetch(0);
      for (int t0 = 0; t0 < tmax; t0 += PD) {
        int jc[PD];
        float rc[PD];
        sfor<0, PD>([&](auto E) {
          jc[E] = jn[E];
          rc[E] = rn[E];
        });
        if (t0 + PD < tmax) fetch(t0 + PD);
        sfor<0, PD>([&](auto E) {
          const int t = t0 + (int)E;
          if (t < tmax) {  // wave-uniform
            const bool ok = t < cnt;
            int j = jc[E];
            const float r0 = rc[E];
            if (ok && (j < 0 || j >= n)) pflags |= 2;
            if (ok && !__builtin_isfinite(r0)) pflags |= 1;
            j = (ok && j >= 0 && j < n) ? j : -1;
            const float r = j >= 0 ? r0 : 0.f;
            float a[N];
            sfor<0, N>([&](auto J) { a[J] = Fr.row1(j, 4 * J + qi); });
            sfor<0, N>([&](auto I) {
              sfor<0, I + 1>([&](auto J) {
                if constexpr (ROW)
                  acc[tri(I, J)] = mfma4x4(a[J], a[I], acc[tri(I, J)]);
                else
                  acc[tri(I, J)] = mfma4x4(a[I], a[J], acc[tri(I, J)]);
              });
            });
            sfor<0, N>([&](auto J) { pb[J] = __builtin_fmaf(r, a[J], pb[J]); });
          }
        });
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // ridge term (unit diagonal on padded rows of a dual system)
    const float reg = lambda * (weighted ? (float)cnt : 1.0f);
    sfor<0, N>([&](auto J) {
      const int c = 4 * J + qi;
      const float dg = (!DUAL || c < cnt) ? reg : 1.0f;
      sfor<0, 4>([&](auto v) { acc[tri(J, J)][(int)v] += (qi == (int)v) ? dg : 0.f; });
    });
    if constexpr (ROW) {
      sfor<0, N>([&](auto I) {
        sfor<0, I + 1>([&](auto J) {
          sfor<0, 4>([&](auto v) { st[I][4 * J + v] = acc[tri(I, J)][(int)v]; });
        });
      });
    } else if constexpr (P == 4) {
      // the MFMA layout already is the owned-column layout
      sfor<0, M>([&](auto m) {
        sfor<0, D>([&](auto j) {
          constexpr int r = 4 * decltype(m)::value + decltype(j)::value;
          if constexpr (r < D) st[m][j] = acc[tri(r / 4, decltype(m)::value)][r % 4];
        });
      });
    } else {
      // lower triangle of each system to LDS, then the system's P lanes read their columns
      float *sys = tri_buf + (lane >> 2) * ST;
      sfor<0, N>([&](auto I) {
        sfor<0, I + 1>([&](auto J) {
          sfor<0, 4>([&](auto v) {
            const int r = 4 * I + (int)v, c = 4 * J + qi;
            if (r >= c) sys[r * (r + 1) / 2 + c] = acc[tri(I, J)][(int)v];
          });
        });
      });
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (sme / 16 == sb) {
        const float *mine = tri_buf + (sme % 16) * ST;
        sfor<0, M>([&](auto m) {
          sfor<0, D>([&](auto j) {
            constexpr int mm = decltype(m)::value, jj = decltype(j)::value;
            if constexpr (P * mm + jj < D) {
              const int r = P * mm + jj, c = P * mm + pi;
              const int hi = r > c ? r : c, lo = r > c ? c : r;
              st[mm][jj] = mine[hi * (hi + 1) / 2 + lo];
            }
          });
        });
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }

  // ---- right-hand side, owned like the columns: lane pi holds bm[m] = b[P m + pi]
  float bm[M];
  if constexpr (DUAL) {
    sfor<0, M>([&](auto m) { bm[m] = vxs[sme * E + P * m + pi]; });
  } else {
    // b = F_O^T r in the quad layout: lane q of the quad holds b[4J + q], the owned layout
    static_assert(DUAL || P == 4, "primal systems use four lanes");
    sfor<0, M>([&](auto m) { bm[m] = pb[m]; });
    my_flags |= pflags;
  }

  // ---- elimination with fused forward substitution
  int bad = 0;
  if constexpr (BLK) {
    // Blocked by tile columns (four lanes per system).  The four pivots of tile column t update
    // only that tile column (the panel); the trailing tiles then get the rank-4 update
    //   G[4I+i][4J+j] -= sum_q Gp[4I+i][4t+q] Gp[4J+j][4t+q] / d_q   (I >= J > t)
    // on MFMA, Gp being the panel column at its pivot.  The instruction needs row i of a
    // panel tile in lane i; four MFMAs against unit vectors transpose a tile in the quad.
    static_assert(P == 4 && DUAL, "the blocked elimination works on the four-lane dual layout");
    sfor<0, N>([&](auto Tt) {
      constexpr int t = decltype(Tt)::value;
      float sv[4], tyv[4];  // 1 / d_q and -b_q / d_q of the tile's pivots
      sfor<0, 4>([&](auto PPp) {
        constexpr int pp = decltype(PPp)::value, p = 4 * t + pp;
        const float d = quad_bcast_c<pp>(st[t][pp]);
        bad |= !(d > 0.f);
        const float sp = __builtin_amdgcn_rcpf(d);
        const float ty = -sp * quad_bcast_c<pp>(bm[t]);
        sv[pp] = sp;
        tyv[pp] = ty;
        float g[D];
        sfor<p + 1, D>([&](auto R) {
          constexpr int r = decltype(R)::value;
          g[r] = quad_bcast_c<pp>(st[t][r - 4 * t]);
        });
        float cand[4];
        sfor<0, 4>([&](auto k) {
          constexpr int c = 4 * t + decltype(k)::value;
          if constexpr (c > p)
            cand[k] = g[c];
          else
            cand[k] = 0.f;
        });
        const float go = pick<4>(cand, pi);
        bm[t] = __builtin_fmaf(go, ty, bm[t]);
        if constexpr (pp < 3) {
          const float lc = go * (-sp);
          sfor<p + 1, D>([&](auto R) {
            constexpr int r = decltype(R)::value;
            st[t][r - 4 * t] = __builtin_fmaf(g[r], lc, st[t][r - 4 * t]);
          });
        }
      });
      if constexpr (t + 1 < N) {
        f4 tt[N], ts[N];  // transposed panel tiles (lane = row, register = panel column), scaled copy
        sfor<t + 1, N>([&](auto Ii) {
          constexpr int I = decltype(Ii)::value;
          f4 x = f4{0.f, 0.f, 0.f, 0.f};
          sfor<0, 4>([&](auto S) {
            constexpr int s_ = decltype(S)::value;
            x = mfma4x4(st[t][4 * (I - t) + s_], qi == s_ ? 1.f : 0.f, x);
          });
          tt[I] = x;
          f4 y;
          sfor<0, 4>([&](auto q) {
            y[(int)q] = x[(int)q] * (-sv[q]);
            bm[I] = __builtin_fmaf(x[(int)q], tyv[q], bm[I]);  // trailing right-hand side
          });
          ts[I] = y;
        });
        sfor<t + 1, N>([&](auto Ii) {
          constexpr int I = decltype(Ii)::value;
          sfor<t + 1, I + 1>([&](auto Jj) {
            constexpr int J = decltype(Jj)::value, o = 4 * (I - J);
            f4 a = f4{st[J][o], st[J][o + 1], st[J][o + 2], st[J][o + 3]};
            sfor<0, 4>([&](auto q) { a = mfma4x4(tt[I][(int)q], ts[J][(int)q], a); });
            sfor<0, 4>([&](auto v) { st[J][o + v] = a[(int)v]; });
          });
        });
      }
    });
  } else if constexpr (ROW) {
    sfor<0, D>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value, mp = p / 4, pp = p % 4;
      constexpr int m0 = pp == 3 ? mp + 1 : mp;  // first tile with rows below the pivot
      const float d = quad_bcast_c<pp>(st[mp][p]);
      bad |= !(d > 0.f);
      const float s = __builtin_amdgcn_rcpf(d);
      const float zp = quad_bcast_c<pp>(bm[mp]) * s;  // z_p = y_p / d_p
      // the lane's rows c = 4I + pi below the pivot: G[c][p] (zero for c <= p), the forward
      // substitution, and -L[c][p] = -G[c][p] / d_p kept in place for the back substitution
      float gc[M];
      sfor<m0, M>([&](auto Ii) {
        constexpr int I = decltype(Ii)::value;
        float v = st[I][p];
        if constexpr (I == mp) v = pi > pp ? v : 0.f;
        gc[I] = v;
        bm[I] = __builtin_fmaf(-v, zp, bm[I]);
        st[I][p] = -v * s;
      });
      bm[mp] = pi == pp ? zp : bm[mp];
      // trailing update G[c][j] += G[c][p] (-G[j][p] / d_p) for c, j > p.  Tile column m0, which
      // holds the next pivot's column, on the VALU: the factor of column j comes from row j's
      // lane by DPP (rows of the diagonal tile above c are updated too, unused).
      if constexpr (m0 < M) {
        sfor<(p + 1 > 4 * m0 ? p + 1 : 4 * m0), 4 * m0 + 4>([&](auto Jj) {
          constexpr int j = decltype(Jj)::value;
          const float lj = quad_bcast_c<j % 4>(st[m0][p]);
          sfor<m0, M>([&](auto Ii) {
            constexpr int I = decltype(Ii)::value;
            st[I][j] = __builtin_fmaf(gc[I], lj, st[I][j]);
          });
        });
      }
      // Later tile columns, needed a pivot or more later, as one rank-1 MFMA per tile (I, J):
      // register v of lane q is G[4I + q][4J + v], so the A operand is the factor of rows
      // 4J .. 4J + 3 (lane v's own st[J][p]) and the B operand the lane's gc[I].
      sfor<m0 + 1, M>([&](auto Jj) {
        constexpr int J = decltype(Jj)::value;
        const float lJ = st[J][p];
        sfor<J, M>([&](auto Ii) {
          constexpr int I = decltype(Ii)::value;
          f4 t = f4{st[I][4 * J], st[I][4 * J + 1], st[I][4 * J + 2], st[I][4 * J + 3]};
          t = mfma4x4(lJ, gc[I], t);
          sfor<0, 4>([&](auto v) { st[I][4 * J + v] = t[(int)v]; });
        });
      });
    });
  } else {
    sfor<0, D>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value, mp = p / P, pp = p % P;
      const float d = grp_bcast<P, pp>(st[mp][pp]);
      bad |= !(d > 0.f);
      const float s = __builtin_amdgcn_rcpf(d);
      const float ty = -s * grp_bcast<P, pp>(bm[mp]);  // -b[p] / d
      if constexpr (P == 1) {
        // the pivot column is the lane's own: update every later column
        sfor<p + 1, D>([&](auto C) {
          constexpr int c = decltype(C)::value;
          const float lc = st[mp][c - mp] * (-s);  // -G[c][p] / d
          bm[c] = __builtin_fmaf(st[mp][c - mp], ty, bm[c]);
          sfor<c, D>([&](auto R) {
            constexpr int r = decltype(R)::value;
            st[c][r - c] = __builtin_fmaf(st[mp][r - mp], lc, st[c][r - c]);
          });
        });
      } else {
        // column p below the pivot, broadcast from its owner lane: g[r] = G[r][p]
        float g[D];
        sfor<p + 1, D>([&](auto R) {
          constexpr int r = decltype(R)::value;
          g[r] = grp_bcast<P, pp>(st[mp][r - P * mp]);
        });
        // owned columns c = P m + pi: multiplier -G[c][p] / d and rhs, no-ops for c <= p
        float lc[M];
        sfor<mp, M>([&](auto Mm) {
          constexpr int m = decltype(Mm)::value;
          float cand[P];
          sfor<0, P>([&](auto k) {
            constexpr int c = P * m + decltype(k)::value;
            if constexpr (c > p)
              cand[k] = g[c];
            else
              cand[k] = 0.f;
          });
          const float go = pick<P>(cand, pi);
          lc[m] = go * (-s);
          bm[m] = __builtin_fmaf(go, ty, bm[m]);
        });
        // the pivot's own tile column is finished when p is its last column (lc = 0 there)
        constexpr int m0 = pp == P - 1 ? mp + 1 : mp;
        sfor<p + 1, D>([&](auto R) {
          constexpr int r = decltype(R)::value;
          sfor<m0, (r / P + 1 < M ? r / P + 1 : M)>([&](auto Mm) {
            constexpr int m = decltype(Mm)::value;
            st[m][r - P * m] = __builtin_fmaf(g[r], lc[m], st[m][r - P * m]);
          });
        });
      }
    });
  }

  // ---- back substitution; dot[m] accumulates sum_{r > c} G[r][c] x_r for owned column c.
  // Dual systems fold each x_p into u = F_O^T x as soon as it is known: lane pi forms the
  // outputs [pi K/P, (pi+1) K/P).  Primal systems keep x in the owned layout.
  constexpr int KO = K / P;
  static_assert(!DUAL || KO % 4 == 0, "dual outputs are formed in 4-float chunks per lane");
  f4 u[DUAL ? KO / 4 : 1];
  if constexpr (DUAL) sfor<0, KO / 4>([&](auto c) { u[c] = f4{0.f, 0.f, 0.f, 0.f}; });
  if constexpr (ROW) {
    // x_p = z_p - sum_{c > p} L[c][p] x_c: each lane sums over its solved rows (x = 0 until a
    // row is solved), then the quad adds its four partial sums
    float xv[M];
    sfor<0, M>([&](auto m) { xv[m] = 0.f; });
    sfor_down<0, D>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value, mp = p / 4, pp = p % 4;
      float part = st[mp][p] * xv[mp];
      sfor<mp + 1, M>([&](auto Ii) {
        constexpr int I = decltype(Ii)::value;
        part = __builtin_fmaf(st[I][p], xv[I], part);
      });
      part += quad_xor1(part);
      part += quad_xor2(part);
      const float xp = quad_bcast_c<pp>(bm[mp]) + part;
      xv[mp] = pi == pp ? xp : xv[mp];
      if constexpr (DUAL) {
        const int j = ixs[sme * E + p];
        sfor<0, KO / 4>([&](auto c) { u[c] += xp * Fr.row4(j, pi * KO + 4 * c); });
        if constexpr (D >= 20) __builtin_amdgcn_sched_barrier(0);
      }
    });
    if constexpr (!DUAL) sfor<0, M>([&](auto m) { bm[m] = xv[m]; });
  } else {
    float dot[M];
    sfor<0, M>([&](auto m) { dot[m] = 0.f; });
    sfor_down<0, D>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value, mp = p / P, pp = p % P;
      const float d = grp_bcast<P, pp>(st[mp][pp]);
      const float xo = (bm[mp] - dot[mp]) * __builtin_amdgcn_rcpf(d);  // x_p in its owner lane
      const float xp = grp_bcast<P, pp>(xo);
      sfor<0, mp + 1>([&](auto Mm) {
        constexpr int m = decltype(Mm)::value;
        dot[m] = __builtin_fmaf(st[m][p - P * m], xp, dot[m]);  // row p of owned column P m + pi
      });
      if constexpr (DUAL) {
        const int j = ixs[sme * E + p];
        sfor<0, KO / 4>([&](auto c) { u[c] += xp * Fr.row4(j, pi * KO + 4 * c); });
        // keep the factor-row reads of later pivots from being hoisted here (register pressure)
        if constexpr (D >= 20) __builtin_amdgcn_sched_barrier(0);
      } else {
        if constexpr (P == 1)
          bm[mp] = xo;
        else
          bm[mp] = pi == pp ? xo : bm[mp];
      }
    });
  }

  if constexpr (P == 2) my_flags |= __builtin_amdgcn_mov_dpp(my_flags, 0xb1, 0xf, 0xf, true);
  if constexpr (P == 4) {
    my_flags |= quad_xor1_i(my_flags);
    my_flags |= quad_xor2_i(my_flags);
  }
  const bool good = my_row >= 0 && my_cnt > 0 && !bad && my_flags == 0;
  if (my_row >= 0) {
    if constexpr (DUAL) {
      float *out = X + my_row * K + pi * KO;
      sfor<0, KO / 4>([&](auto c) { *reinterpret_cast<f4 *>(out + 4 * c) = good ? u[c] : f4{0.f, 0.f, 0.f, 0.f}; });
    } else {
      sfor<0, M>([&](auto m) { X[my_row * K + P * m + pi] = good ? bm[m] : 0.f; });
    }
  }
  if (status && my_row >= 0 && pi == 0)
    status[my_row] = my_cnt == 0      ? OPEN_ROW_EMPTY
                     : (my_flags & 2) ? OPEN_ROW_BADINDEX
                     : (my_flags & 1) ? OPEN_ROW_NONFINITE
                     : bad            ? OPEN_ROW_NONPOS_PIVOT
                                      : OPEN_ROW_OK;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();  // the group's LDS lists are reused by the next group
}

// LDS budget of a block (bytes) and the factor matrix staged beside the per-wave buffers.
constexpr int kLdsBytes = 160 * 1024;
constexpr int kFactorLdsRows = 512;  // factor rows a block can stage (the fold-in has 480)
// the zero row, kFactorLdsRows rows at pitch K + 4, and one wave instruction (64 slots) of tail
template <int K>
__host__ __device__ constexpr int factor_lds_bytes() { return ((kFactorLdsRows + 1) * (K + 4) + 256) * 4; }
template <int K, int P, int D>
__host__ __device__ constexpr int wave_bytes() { return wave_lds_floats(P, D) * 4; }

// Persistent kernel over the rows of classes c_lo..c_hi (contiguous in the bucketed list),
// all solved at padded dimension D (dual) or k (primal).
template <int K, int P, int D, bool DUAL, bool LDSF, int W, int OCC, bool BLK>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * W, 64 * W), amdgpu_waves_per_eu(OCC))) void k_solve_class(const float *__restrict__ F, int n,
                                                     const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                     const float *__restrict__ val, const RowRef *__restrict__ list,
                                                     const int64_t *__restrict__ cls, int c_lo, int c_hi, float lambda,
                                                     int weighted, float *__restrict__ X,
                                                     int32_t *__restrict__ status) {
  constexpr int SYS = 64 / P;
  constexpr int WL = wave_lds_floats(P, D);
  constexpr int FL = LDSF ? factor_lds_bytes<K>() / 4 : 4;
  __shared__ __attribute__((aligned(16))) float lds_all[W * WL + FL];
  const int64_t start = cls[2 * c_lo];
  const int64_t count = cls[2 * c_hi] + cls[2 * c_hi + 1] - start;
  const int64_t end = start + count;
  const int64_t nw = (int64_t)gridDim.x * W;
  const int64_t g0 = (int64_t)blockIdx.x * W + (threadIdx.x >> 6);
  if ((int64_t)blockIdx.x * W * SYS >= count) return;  // block has no work (uniform)
  FRows<K, LDSF> Fr;
  if constexpr (LDSF) {
    // [zero row][n rows at pitch PS][tail]: direct global -> LDS copies, one 16-byte slot
    // per lane and 1 KB per wave instruction; a row's pad slot copies its chunk 0, and the
    // lanes of the last instruction past the end copy the last chunk into the tail
    constexpr int PS = K + 4, CH = K / 4, SL = CH + 1;
    float *fl = lds_all + W * WL;
    const int slots = n * SL;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int base = w * 64; base < slots; base += W * 64) {
      const int e = base + lane < slots ? base + lane : slots - 2;  // slots - 2: last data chunk
      const int jj = e / SL, cc = e % SL;
      __builtin_amdgcn_global_load_lds(F + (int64_t)jj * K + 4 * (cc < CH ? cc : 0),
                                       (__attribute__((address_space(3))) void *)(fl + PS + 4 * base), 16, 0, 0);
    }
    if (threadIdx.x < PS) fl[threadIdx.x] = 0.f;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    Fr.lds = fl + PS;
  } else {
    Fr.rs = make_rsrc(F, (uint64_t)n * K * sizeof(float));
  }
  float *wl = lds_all + (threadIdx.x >> 6) * WL;
  const int sme = (threadIdx.x & 63) / P;
  auto fetch = [&](int64_t g) -> RowRef {
    const int64_t sl = start + g * SYS + sme;
    return (g * SYS < count && sl < end) ? list[sl] : RowRef{-1, 0, 0};
  };
  RowRef cur = fetch(g0);
  for (int64_t g = g0; g * SYS < count; g += nw) {
    const RowRef nxt = fetch(g + nw);  // next group's records load while this group computes
    // operand prefetch in the Gram loop when a single wave per SIMD has to hide the latency
    solve_group<P, D, K, DUAL, LDSF, (OCC == 1 || D <= 12), BLK>(Fr, n, cur, idx, val, lambda, weighted, X, status,
                                                                 wl);
    cur = nxt;
  }
}

// ---------------------------------------------------------------- several classes, one launch
// A size class inside a merged launch: padded dimension D (k for the primal form), the form,
// and its classes c_lo..c_hi of the bucketed list.
template <int D_, bool DUAL_, int CLO_, int CHI_>
struct SizeClass {
  static constexpr int D = D_, CLO = CLO_, CHI = CHI_;
  static constexpr bool DUAL = DUAL_;
};

template <int P, typename... C>
__host__ __device__ constexpr int multi_wave_floats() {
  int m = 0;
  ((m = wave_lds_floats(P, C::D) > m ? wave_lds_floats(P, C::D) : m), ...);
  return m;
}

// Persistent kernel over the rows of several size classes that share one launch shape (P lanes
// per system, W waves per block, OCC waves per SIMD): the groups of 64 / P systems of the
// classes, in the order given (the costliest first, so that the cheap ones fill the tail), are
// one index space that the waves stride through.  Each group is solved exactly as by the
// class's own kernel.
template <int K, int P, bool LDSF, int W, int OCC, typename... C>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * W, 64 * W), amdgpu_waves_per_eu(OCC))) void k_solve_multi(
    const float *__restrict__ F, int n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
    const float *__restrict__ val, const RowRef *__restrict__ list, const int64_t *__restrict__ cls, float lambda,
    int weighted, float *__restrict__ X, int32_t *__restrict__ status) {
  constexpr int NC = sizeof...(C);
  constexpr int SYS = 64 / P;
  constexpr int WL = multi_wave_floats<P, C...>();
  constexpr int FL = LDSF ? factor_lds_bytes<K>() / 4 : 4;
  __shared__ __attribute__((aligned(16))) float lds_all[W * WL + FL];
  // per class: first list slot, rows, and the first group of the merged index space
  int64_t cs[NC], cc[NC], g1[NC];
  {
    int i = 0;
    int64_t acc = 0;
    ((cs[i] = cls[2 * C::CLO], cc[i] = cls[2 * C::CHI] + cls[2 * C::CHI + 1] - cs[i], acc += (cc[i] + SYS - 1) / SYS,
      g1[i] = acc, ++i),
     ...);
  }
  const int64_t total = g1[NC - 1];  // groups of all classes
  const int64_t nw = (int64_t)gridDim.x * W;
  (void)ptr;
  const int64_t g0 = (int64_t)blockIdx.x * W + (threadIdx.x >> 6);
  if ((int64_t)blockIdx.x * W >= total) return;  // block has no work (uniform)
  FRows<K, LDSF> Fr;
  if constexpr (LDSF) {
    constexpr int PS = K + 4, CH = K / 4, SL = CH + 1;
    float *fl = lds_all + W * WL;
    const int slots = n * SL;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int base = w * 64; base < slots; base += W * 64) {
      const int e = base + lane < slots ? base + lane : slots - 2;  // slots - 2: last data chunk
      const int jj = e / SL, cc2 = e % SL;
      __builtin_amdgcn_global_load_lds(F + (int64_t)jj * K + 4 * (cc2 < CH ? cc2 : 0),
                                       (__attribute__((address_space(3))) void *)(fl + PS + 4 * base), 16, 0, 0);
    }
    if (threadIdx.x < PS) fl[threadIdx.x] = 0.f;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    Fr.lds = fl + PS;
  } else {
    Fr.rs = make_rsrc(F, (uint64_t)n * K * sizeof(float));
  }
  float *wl = lds_all + (threadIdx.x >> 6) * WL;
  const int sme = (threadIdx.x & 63) / P;
  // The wave takes the merged groups g = g0 (mod nw) in increasing order: one loop per class,
  // over the class's own groups, so that each loop holds only its class's registers.
  int ci = 0;
  (
      [&] {
        const int i = ci++;
        const int64_t gb = i ? g1[i - 1] : 0;  // first merged group of the class
        const int64_t ng = g1[i] - gb;
        int64_t gl = (g0 - gb) % nw;           // the wave's first group of the class
        if (gl < 0) gl += nw;
        auto fetch = [&](int64_t q) -> RowRef {
          const int64_t sl = q * SYS + sme;
          return (q < ng && sl < cc[i]) ? list[cs[i] + sl] : RowRef{-1, 0, 0};
        };
        RowRef cur = fetch(gl);
        for (int64_t q = gl; q < ng; q += nw) {
          const RowRef nxt = fetch(q + nw);  // next group's records load while this group computes
          solve_group<P, C::D, K, C::DUAL, LDSF, (OCC == 1 || C::D <= 12), false>(Fr, n, cur, idx, val, lambda,
                                                                                  weighted, X, status, wl);
          cur = nxt;
        }
      }(),
      ...);
}

template <int K, int P, int W, int OCC, typename... C>
open_status launch_multi(const char *name, open_ctx *ctx, const float *F, int n, const int64_t *ptr,
                         const int32_t *idx, const float *val, float lambda, int weighted, const RowRef *list,
                         const int64_t *cls, float *X, int32_t *status, int64_t m) {
  const int64_t groups = (m + 64 / P - 1) / (64 / P) + (int64_t)sizeof...(C);
  int64_t blocks = (groups + W - 1) / W;
  constexpr int waves_b = W * multi_wave_floats<P, C...>() * 4;
  constexpr int flb = factor_lds_bytes<K>();
  constexpr bool fl_fits = waves_b + flb <= kLdsBytes;
  static_assert(waves_b + 16 <= kLdsBytes, "per-wave buffers exceed LDS");
  const bool fl = fl_fits && n <= kFactorLdsRows;
  const int lds_cu = kLdsBytes / (waves_b + (fl ? flb : 16));
  const int reg_cu = 4 * OCC / W;
  int per_cu = lds_cu < reg_cu ? lds_cu : reg_cu;
  const int64_t cap = (int64_t)ctx->num_cu * (per_cu < 1 ? 1 : per_cu);
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  if constexpr (fl_fits) {
    if (fl) {
      OPEN_LAUNCH(ctx, name, (k_solve_multi<K, P, true, W, OCC, C...>), dim3((unsigned)blocks), dim3(64 * W), 0, F, n,
                  ptr, idx, val, list, cls, lambda, weighted, X, status);
      return OPEN_OK;
    }
  }
  OPEN_LAUNCH(ctx, name, (k_solve_multi<K, P, false, W, OCC, C...>), dim3((unsigned)blocks), dim3(64 * W), 0, F, n,
              ptr, idx, val, list, cls, lambda, weighted, X, status);
  return OPEN_OK;
}

// Launch the kernel of one size class with a persistent grid sized for m rows: blocks of W
// waves (sharing one LDS copy of the factors), as many per CU as LDS and the register
// budget of OCC waves per SIMD allow.
template <int K, int P, int D, bool DUAL, int W = 4, int OCC = 1, bool BLK = false>
open_status launch_class(const char *name, open_ctx *ctx, const float *F, int n, const int64_t *ptr,
                         const int32_t *idx, const float *val, float lambda, int weighted, const RowRef *list,
                         const int64_t *cls, int c_lo, int c_hi, float *X, int32_t *status, int64_t m) {
  static_assert(W >= 1 && W <= 16 && OCC >= 1 && OCC <= 8, "block shape");
  const int64_t groups = (m + 64 / P - 1) / (64 / P);
  int64_t blocks = (groups + W - 1) / W;
  constexpr int waves_b = W * wave_bytes<K, P, D>();
  constexpr int flb = factor_lds_bytes<K>();
  constexpr bool fl_fits = waves_b + flb <= kLdsBytes;
  static_assert(waves_b + 16 <= kLdsBytes, "per-wave buffers exceed LDS");
  // stage the factors in LDS when they fit beside the per-wave buffers
  const bool fl = fl_fits && n <= kFactorLdsRows;
  const int lds_cu = kLdsBytes / (waves_b + (fl ? flb : 16));
  const int reg_cu = 4 * OCC / W;  // waves a CU holds at OCC per SIMD, in blocks
  int per_cu = lds_cu < reg_cu ? lds_cu : reg_cu;
  const int64_t cap = (int64_t)ctx->num_cu * (per_cu < 1 ? 1 : per_cu);
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  if constexpr (fl_fits) {
    if (fl) {
      OPEN_LAUNCH(ctx, name, (k_solve_class<K, P, D, DUAL, true, W, OCC, BLK>), dim3((unsigned)blocks), dim3(64 * W), 0,
                  F, n, ptr, idx, val, list, cls, c_lo, c_hi, lambda, weighted, X, status);
      return OPEN_OK;
    }
  }
  OPEN_LAUNCH(ctx, name, (k_solve_class<K, P, D, DUAL, false, W, OCC, BLK>), dim3((unsigned)blocks), dim3(64 * W), 0, F,
              n, ptr, idx, val, list, cls, c_lo, c_hi, lambda, weighted, X, status);
  return OPEN_OK;
}

#define OPEN_TIER_ARGS                                                                                    \
  open_ctx *ctx, const float *F, int n, const int64_t *ptr, const int32_t *idx, const float *val, float lambda, \
      int weighted, const RowRef *list, const int64_t *cls, float *X, int32_t *status, int64_t m
#define OPEN_TIER_PASS ctx, F, n, ptr, idx, val, lambda, weighted, list, cls

// ---------------------------------------------------------------- kernel variants
// A kernel configuration in one integer: P lanes per system, W waves per block, OCC waves per
// SIMD that the register allocation must allow, and BLK for the blocked (MFMA trailing
// update) elimination.
constexpr int cfg(int P, int W, int OCC, int BLK = 0) { return BLK * 1000000 + P * 10000 + W * 100 + OCC; }

// Launch configuration number `choice` of C... for one class group.
template <int K, int D, bool DUAL, int... C>
open_status launch_variant(int choice, const char *name, int c_lo, int c_hi, OPEN_TIER_ARGS) {
  open_status st = OPEN_OK;
  int i = 0;
  bool done = false;
  ((i++ == choice ? (void)(done = true, st = launch_class<K, (C / 10000) % 100, D, DUAL, (C / 100) % 100, C % 100, (C / 1000000) != 0>(
                                            name, OPEN_TIER_PASS, c_lo, c_hi, X, status, m))
                  : (void)0),
   ...);
  if (!done) return fail(ctx, OPEN_E_INVALID, "kernel variant out of range");
  return st;
}

// A group of size classes solved by one kernel, with its compiled variants.
using group_fn = open_status (*)(int choice, OPEN_TIER_ARGS);
struct ClassGroup {
  const char *name;
  int c_lo, c_hi;  // classes of the bucketed list it covers
  int nvar;        // configurations compiled (variant 0 is the default)
  group_fn fn;
};

// The class groups of rank k (8, 16, 32 or 64) and their number; nullptr for other ranks.
const ClassGroup *class_groups(int k, int *count);

#define OPEN_GROUP(NAME) open_status NAME(int choice, OPEN_TIER_ARGS)
// The rank-32 pass in three merged launches, selected by the launch-mode entry of the rank's
// tuning table (0: merged, 1: one launch per class group).
open_status rowsolve_k32_merged(OPEN_TIER_ARGS);
OPEN_GROUP(g_k8_d4);
OPEN_GROUP(g_k8_d8);
OPEN_GROUP(g_k8_primal);
OPEN_GROUP(g_k16_d4);
OPEN_GROUP(g_k16_d8);
OPEN_GROUP(g_k16_d12);
OPEN_GROUP(g_k16_d16);
OPEN_GROUP(g_k16_primal);
OPEN_GROUP(g_k32_d4);
OPEN_GROUP(g_k32_d8);
OPEN_GROUP(g_k32_d12);
OPEN_GROUP(g_k32_d16);
OPEN_GROUP(g_k32_d20);
OPEN_GROUP(g_k32_d24);
OPEN_GROUP(g_k32_d28);
OPEN_GROUP(g_k32_d32);
OPEN_GROUP(g_k32_primal);
OPEN_GROUP(g_k64_d4);
OPEN_GROUP(g_k64_d8);
OPEN_GROUP(g_k64_d12);
OPEN_GROUP(g_k64_d16);
OPEN_GROUP(g_k64_d20);
OPEN_GROUP(g_k64_d24);
OPEN_GROUP(g_k64_d28);
OPEN_GROUP(g_k64_d32);
OPEN_GROUP(g_k64_primal);

}  // namespace openk
