// Rank-64 ridge solves of rows with more than 32 observed entries (the primal form of the
// fold-in and of the ALS row half-sweep, Section III-B.2, with the ALS-WR weighting of the
// paper's CF reference):
//     (sum_{j in O_i} f_j f_j^T + lambda w_i I_64) u_i = sum_{j in O_i} r_ij f_j.
// The 64 x 64 system of a row does not fit the register layouts of the other size classes, so
// each row gets one wavefront:
//   Gram   the row's entries are staged in LDS (1024 per chunk); the factor rows are gathered
//          through a bounds-checked buffer resource (index -1 of padding reads zero), two
//          observations per v_mfma_f32_32x32x2f32 step, three 32x32 blocks (A11, A21, A22) in
//          float32 accumulators; the right-hand side accumulates beside them.
//   Layout the blocks go to LDS as the full symmetric matrix (pitch 65, conflict-free columns)
//          with the ridge on the diagonal; lane c then holds column c in 64 registers.
//   Solve  right-looking LDL^T without pivoting (SPD): at pivot p every lane writes its entry
//          of row p of the (symmetric) trailing matrix to LDS, and every lane reads the row
//          back as 16-byte broadcasts, which is column p below the pivot; lane c applies the
//          multiplier A[p][c] / d_p to its rows r > p and to its right-hand side (forward
//          substitution fused in).  After the elimination lane r still holds d_r L[p][r] in
//          register p > r, so the back substitution is column-oriented: x_p is broadcast
//          with a lane read and lanes r < p subtract d_r L[p][r] x_p.
//   Output lane c writes u_c (one 256-byte row per wavefront).
#include "rowsolve.h"

namespace openk {

constexpr int kP64Waves = 4;                 // wavefronts per block
constexpr int kP64Pitch = 65;                // LDS pitch of the 64 x 64 matrix
constexpr int kP64Mat = 64 * kP64Pitch;      // matrix floats per wavefront
constexpr int kP64Chunk = 1024;              // entries staged per chunk (indices + values)
constexpr int kP64Unr = 8;                   // MFMA steps (2 observations each) per batch
static_assert(2 * kP64Chunk <= kP64Mat, "entry staging aliases the matrix area");

typedef float f16v __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(64 * kP64Waves) __attribute__((amdgpu_waves_per_eu(2))) void k_primal64(const float *__restrict__ F, int n,
                                                             const int32_t *__restrict__ idx,
                                                             const float *__restrict__ val,
                                                             const RowRef *__restrict__ list,
                                                             const int64_t *__restrict__ cls, int c_lo, int c_hi,
                                                             float lambda, int weighted, float *__restrict__ X,
                                                             int32_t *__restrict__ status) {
  __shared__ __attribute__((aligned(16))) float lds[kP64Waves][kP64Mat + 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float *mat = lds[w];
  float *colb = lds[w] + kP64Mat;  // pivot column broadcast buffer
  int *jl = reinterpret_cast<int *>(mat);
  float *rl = mat + kP64Chunk;
  const int64_t start = cls[2 * c_lo];
  const int64_t count = cls[2 * c_hi] + cls[2 * c_hi + 1] - start;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(F, (uint64_t)n * 64 * sizeof(float));
  const int d = lane & 31, o = lane >> 5;  // dimension and observation slot in an MFMA step
  const int64_t nw = (int64_t)gridDim.x * kP64Waves;
  for (int64_t g = (int64_t)blockIdx.x * kP64Waves + w; g < count; g += nw) {
    const RowRef rr = list[start + g];
    f16v a11 = f16v{}, a21 = f16v{}, a22 = f16v{};
    float bl = 0.f, bh = 0.f;
    int flags = 0;  // 1: non-finite value, 2: column index outside [0, n)
    for (int c0 = 0; c0 < rr.cnt; c0 += kP64Chunk) {
      const int len = rr.cnt - c0 < kP64Chunk ? rr.cnt - c0 : kP64Chunk;
      const int lenp = (len + 2 * kP64Unr - 1) & ~(2 * kP64Unr - 1);  // <= kP64Chunk
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the previous chunk's (or row's) LDS reads are done
      for (int t = lane; t < lenp; t += 64) {
        const bool in = t < len;
        const int j = in ? idx[rr.beg + c0 + t] : -1;
        const float r = in ? val[rr.beg + c0 + t] : 0.f;
        const bool jok = j >= 0 && j < n;
        if (in && !jok) flags |= 2;
        if (in && !__builtin_isfinite(r)) flags |= 1;
        jl[t] = jok ? j : -1;
        rl[t] = r;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      float ul[kP64Unr], uh[kP64Unr], rv[kP64Unr];
      auto load = [&](int t0) {
#pragma unroll
        for (int u = 0; u < kP64Unr; ++u) {
          const int t = t0 + 2 * u + o;
          const int j = jl[t];
          rv[u] = rl[t];
          const uint32_t off = (uint32_t)(j * 64 + d) * 4u;  // j = -1 wraps out of range: zero
          ul[u] = bload_f32(rs, (int)off);
          uh[u] = bload_f32(rs, (int)(off + 128u));
        }
      };
      load(0);
      for (int t0 = 0; t0 < lenp; t0 += 2 * kP64Unr) {
        float cl[kP64Unr], ch[kP64Unr], cr[kP64Unr];
#pragma unroll
        for (int u = 0; u < kP64Unr; ++u) {
          cl[u] = ul[u];
          ch[u] = uh[u];
          cr[u] = rv[u];
        }
        if (t0 + 2 * kP64Unr < lenp) load(t0 + 2 * kP64Unr);
#pragma unroll
        for (int u = 0; u < kP64Unr; ++u) {
          a11 = __builtin_amdgcn_mfma_f32_32x32x2f32(cl[u], cl[u], a11, 0, 0, 0);
          a21 = __builtin_amdgcn_mfma_f32_32x32x2f32(ch[u], cl[u], a21, 0, 0, 0);
          a22 = __builtin_amdgcn_mfma_f32_32x32x2f32(ch[u], ch[u], a22, 0, 0, 0);
          bl = __builtin_fmaf(cr[u], cl[u], bl);
          bh = __builtin_fmaf(cr[u], ch[u], bh);
        }
      }
    }
    // ---- the symmetric matrix to LDS: lane l holds column l % 32 of each block, register v
    // row 8 (v / 4) + 4 (l / 32) + v % 4 of it; the A21 block is written on both sides
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the staging area is about to be overwritten
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v / 4) + 4 * o + (v % 4);
      mat[r * kP64Pitch + d] = a11[v];
      mat[(32 + r) * kP64Pitch + d] = a21[v];
      mat[d * kP64Pitch + 32 + r] = a21[v];
      mat[(32 + r) * kP64Pitch + 32 + d] = a22[v];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float reg = lambda * (weighted ? (float)rr.cnt : 1.0f);
    float a[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) a[r] = mat[r * kP64Pitch + lane];
    // ridge on the diagonal: register `lane` of lane `lane`
    {
      int me = lane;
#pragma unroll
      for (int r = 0; r < 64; ++r) {
        asm volatile("" : "+v"(me));
        a[r] += r == me ? reg : 0.f;
      }
    }
    // right-hand side: lanes l and l ^ 32 hold the two observation slots of dimension l % 32
    const float bls = bl + __shfl_xor(bl, 32, 64), bhs = bh + __shfl_xor(bh, 32, 64);
    float b = lane < 32 ? bls : bhs;

    // ---- LDL^T with fused forward substitution
    int bad = 0;
    float dd = 1.f;  // d_lane
    // The lane tests below go through a value the compiler cannot see through, so each step
    // compares afresh instead of keeping 64 precomputed lane masks in scalar registers.
    int me = lane;
    sfor<0, 64>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value, q0 = p / 4;
      asm volatile("" : "+v"(me));
      // row p of the trailing matrix, one entry per lane (register p of lane c is A[p][c]);
      // by symmetry it is also column p below the pivot
      colb[lane] = a[p];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      float gcol[64];
      sfor<q0, 16>([&](auto Q) {
        constexpr int q = decltype(Q)::value;
        const f4 x = *reinterpret_cast<const f4 *>(colb + 4 * q);
        gcol[4 * q] = x[0];
        gcol[4 * q + 1] = x[1];
        gcol[4 * q + 2] = x[2];
        gcol[4 * q + 3] = x[3];
      });
      const float dp = gcol[p];
      bad |= !(dp > 0.f);
      const float inv = __builtin_amdgcn_rcpf(dp);
      const float lc = me > p ? a[p] * inv : 0.f;  // L[c][p] = A[p][c] / d_p for c > p
      sfor<p + 1, 64>([&](auto R) {
        constexpr int r = decltype(R)::value;
        a[r] = __builtin_fmaf(-gcol[r], lc, a[r]);
      });
      const float bp = readlane_f32(b, p);  // y_p, final at step p
      b = __builtin_fmaf(-lc, bp, b);
      dd = me == p ? dp : dd;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the buffer is rewritten at the next pivot
    });
    // ---- back substitution: x_r = (y_r - sum_{p > r} d_r L[p][r] x_p) / d_r
    const float rd = __builtin_amdgcn_rcpf(dd);
    sfor_down<0, 64>([&](auto Pp) {
      constexpr int p = decltype(Pp)::value;
      asm volatile("" : "+v"(me));
      const float xp = readlane_f32(b * rd, p);
      b = me < p ? __builtin_fmaf(-a[p], xp, b) : b;
    });
    const float x = b * rd;
    const bool good = !bad && flags == 0 && rr.cnt > 0;
    X[(int64_t)rr.row * 64 + lane] = good ? x : 0.f;
    const unsigned long long f1 = __ballot(flags & 1), f2 = __ballot(flags & 2);
    if (status && lane == 0)
      status[rr.row] = rr.cnt == 0 ? OPEN_ROW_EMPTY
                       : f2        ? OPEN_ROW_BADINDEX
                       : f1        ? OPEN_ROW_NONFINITE
                       : bad       ? OPEN_ROW_NONPOS_PIVOT
                                   : OPEN_ROW_OK;
  }
}

// The group of size classes 9..15 at rank 64 (n_i > 32 below the split-K length): one
// variant, a persistent grid of up to two blocks per CU (LDS: 4 x 16.9 KB per block).
OPEN_GROUP(g_k64_primal) {
  if (choice != 0) return fail(ctx, OPEN_E_INVALID, "kernel variant out of range");
  int64_t blocks = (m + kP64Waves - 1) / kP64Waves;
  const int64_t cap = (int64_t)ctx->num_cu * 2;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  OPEN_LAUNCH(ctx, "ridge_k64_primal", k_primal64, dim3((unsigned)blocks), dim3(64 * kP64Waves), 0, F, n, idx, val,
              list, cls, 9, 15, lambda, weighted, X, status);
  return OPEN_OK;
}

}  // namespace openk
