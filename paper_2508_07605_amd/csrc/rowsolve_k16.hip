// Ridge-solve tier kernels instantiated in their own translation unit (parallel build).
#include "rowsolve.h"

namespace openk {

open_status tier_k16_dual(OPEN_TIER_ARGS) {
  return launch_tier<16, 1, 4, true>("ridge_k16_dual", OPEN_TIER_PASS, 0, 4, X, status, m);
}

open_status tier_k16_primal(OPEN_TIER_ARGS) {
  return launch_tier<16, 4, 4, false>("ridge_k16_primal", OPEN_TIER_PASS, 9, 15, X, status, m);
}

}  // namespace openk
