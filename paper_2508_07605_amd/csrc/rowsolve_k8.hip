// Ridge-solve tier kernels instantiated in their own translation unit (parallel build).
#include "rowsolve.h"

namespace openk {

open_status tier_k8_dual(OPEN_TIER_ARGS) {
  return launch_tier<8, 1, 2, true>("ridge_k8_dual", OPEN_TIER_PASS, 0, 2, X, status, m);
}

open_status tier_k8_primal(OPEN_TIER_ARGS) {
  return launch_tier<8, 2, 2, false>("ridge_k8_primal", OPEN_TIER_PASS, 9, 15, X, status, m);
}

}  // namespace openk
