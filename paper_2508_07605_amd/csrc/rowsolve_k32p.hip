// Ridge-solve tier kernels instantiated in their own translation unit (parallel build).
#include "rowsolve.h"

namespace openk {

open_status tier_k32_primal(OPEN_TIER_ARGS) {
  return launch_tier<32, 8, 8, false>("ridge_k32_primal", OPEN_TIER_PASS, 9, 15, X, status, m);
}

}  // namespace openk
