// Phase-transition detection (Algorithm 1, Section III-B.2) over many power traces at once.
//
// Algorithm 1 keeps the last N = W / delta GPU power readings (5 s at 0.2 s: N = 25) and
// reports a CPU -> GPU phase transition as soon as none of them is below P_th (60 W); its
// split of the window into 1 s intervals does not change which readings are tested.  The
// report for a trace is therefore the first position t >= N - 1 whose run of consecutive
// readings that are not below P_th, ending at t, is at least N long.
//
// One wavefront per trace (persistent grid), 64 readings per step (one per lane), eight
// steps loaded ahead.  A ballot gives the step's "not below" mask; the run ending at each
// lane is the distance to the last failing reading at or before it (or the carried run plus
// the lane's position when there is none); a second ballot finds the first lane whose run
// reaches N, and the run carried to the next step is read from the step's last lane as a
// scalar.  Reading stops at the report's block of eight steps.
#include "common.h"

namespace openk {

constexpr int kPhaseAhead = 8;

__global__ __launch_bounds__(256) void k_phase_detect(const float *__restrict__ P, int64_t T, int64_t L, int64_t ld,
                                                      float th, int N, int64_t *__restrict__ first) {
  const int lane = threadIdx.x & 63;
  // the wave's index as a scalar, so that the block's buffer resource stays in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t tr = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv; tr < T; tr += nw) {
    const float *row = P + tr * ld;
    int64_t run = 0;  // readings not below the threshold ending just before the current step
    int64_t found = -1;
    for (int64_t base = 0; base < L && found < 0; base += 64 * kPhaseAhead) {
      // the block through a buffer resource: readings past the trace read nothing, and no
      // branch surrounds the loads
      const int64_t rem = L - base;
      const __amdgpu_buffer_rsrc_t rs =
          make_rsrc(row + base, (uint64_t)(rem < 64 * kPhaseAhead ? rem : 64 * kPhaseAhead) * 4);
      float v[kPhaseAhead];
#pragma unroll
      for (int u = 0; u < kPhaseAhead; ++u) v[u] = bload_f32(rs, (64 * u + lane) * 4);
#pragma unroll
      for (int u = 0; u < kPhaseAhead; ++u) {
        const int64_t c0 = base + 64 * u;
        if (c0 >= L || found >= 0) break;  // wave-uniform
        const bool in = c0 + lane < L;
        const bool ok = in && !(v[u] < th);
        const unsigned long long m = __ballot(ok);
        const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const unsigned long long z = ~m & upto;  // failing readings at or before this lane
        const int64_t r = z ? (int64_t)(lane - (63 - __clzll((long long)z))) : run + lane + 1;
        const unsigned long long hit = __ballot(in && r >= N);
        if (hit) {
          found = c0 + __ffsll((long long)hit) - 1;
        } else {
          const int lastl = L - 1 - c0 < 63 ? (int)(L - 1 - c0) : 63;
          run = readlane_i64(r, lastl);  // lastl is wave-uniform
        }
      }
    }
    if (lane == 0) first[tr] = found;
  }
}

}  // namespace openk

using namespace openk;

extern "C" open_status open_phase_detect(open_ctx *ctx, const float *power, int64_t T, int64_t L, int64_t ld,
                                         float threshold, int32_t n_window, int64_t *first_index) {
  if (!ctx) return OPEN_E_INVALID;
  if (T < 0 || L < 0 || ld < L || n_window < 1 || !(threshold == threshold))
    return fail(ctx, OPEN_E_INVALID, "bad shape, window or threshold");
  if (T == 0) return OPEN_OK;
  if (!first_index || (L > 0 && !power)) return fail(ctx, OPEN_E_INVALID, "null pointer");
  OPEN_HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int64_t waves = T < (int64_t)ctx->num_cu * 64 ? T : (int64_t)ctx->num_cu * 64;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  OPEN_LAUNCH(ctx, "phase_detect", k_phase_detect, dim3(blocks), dim3(256), 0, power, T, L, ld, threshold, n_window,
              first_index);
  return OPEN_OK;
}
