// Dispatch of the batched ridge solves to the size-class kernels of each rank.
#include "rowsolve.h"

namespace openk {

open_status rowsolve_launch(open_ctx *ctx, const float *F, int n, int k, const int64_t *ptr, const int32_t *idx,
                            const float *val, float lambda, int weighted, const RowRef *list, const int64_t *cls,
                            float *X, int32_t *status, int64_t m) {
  open_status st = OPEN_OK;
  switch (k) {
    case 8: return classes_k8(OPEN_TIER_PASS, X, status, m);
    case 16: return classes_k16(OPEN_TIER_PASS, X, status, m);
    case 32:
      if ((st = classes_k32_small(OPEN_TIER_PASS, X, status, m))) return st;
      if ((st = classes_k32_mid(OPEN_TIER_PASS, X, status, m))) return st;
      if ((st = classes_k32_large(OPEN_TIER_PASS, X, status, m))) return st;
      return classes_k32_primal(OPEN_TIER_PASS, X, status, m);
    case 64:
      if ((st = classes_k64_small(OPEN_TIER_PASS, X, status, m))) return st;
      if ((st = classes_k64_mid(OPEN_TIER_PASS, X, status, m))) return st;
      return classes_k64_large(OPEN_TIER_PASS, X, status, m);
    default:
      return fail(ctx, OPEN_E_UNSUPPORTED, "rank must be 8, 16, 32 or 64");
  }
}

}  // namespace openk
