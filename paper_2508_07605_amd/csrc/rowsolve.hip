// Dispatch of the batched ridge solves to the tier kernels of each rank.
#include "rowsolve.h"

namespace openk {

open_status rowsolve_launch(open_ctx *ctx, const float *F, int n, int k, const int64_t *ptr, const int32_t *idx,
                            const float *val, float lambda, int weighted, const int32_t *list, const int64_t *cls,
                            float *X, int32_t *status, int64_t m) {
  open_status st = OPEN_OK;
  switch (k) {
    case 8:
      if ((st = tier_k8_dual(OPEN_TIER_PASS, X, status, m))) return st;
      return tier_k8_primal(OPEN_TIER_PASS, X, status, m);
    case 16:
      if ((st = tier_k16_dual(OPEN_TIER_PASS, X, status, m))) return st;
      return tier_k16_primal(OPEN_TIER_PASS, X, status, m);
    case 32:
      if ((st = tier_k32_d14(OPEN_TIER_PASS, X, status, m))) return st;
      if ((st = tier_k32_d56(OPEN_TIER_PASS, X, status, m))) return st;
      if ((st = tier_k32_d78(OPEN_TIER_PASS, X, status, m))) return st;
      return tier_k32_primal(OPEN_TIER_PASS, X, status, m);
    case 64:
      if ((st = tier_k64_d14(OPEN_TIER_PASS, X, status, m))) return st;
      if ((st = tier_k64_d56(OPEN_TIER_PASS, X, status, m))) return st;
      return tier_k64_d78(OPEN_TIER_PASS, X, status, m);
    default:
      return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  }
}

}  // namespace openk
