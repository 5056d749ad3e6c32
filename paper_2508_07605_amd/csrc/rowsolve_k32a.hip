// Ridge-solve tier kernels instantiated in their own translation unit (parallel build).
#include "rowsolve.h"

namespace openk {

open_status tier_k32_d14(OPEN_TIER_ARGS) {
  return launch_tier<32, 1, 4, true>("ridge_k32_d14", OPEN_TIER_PASS, 0, 4, X, status, m);
}

}  // namespace openk
