// Ridge-solve kernels of size-class groups, each with its compiled configurations
// (lanes per system, waves per block, waves per SIMD); variant 0 is the default.
#include "rowsolve.h"

namespace openk {

OPEN_GROUP(g_k8_d4) {
  return launch_variant<8, 4, true, cfg(1, 16, 4), cfg(2, 16, 4)>(choice, "ridge_k8_d4", 0, 1, OPEN_TIER_PASS, X,
                       status, m);
}

OPEN_GROUP(g_k8_d8) {
  return launch_variant<8, 8, true, cfg(1, 16, 4), cfg(2, 16, 4)>(choice, "ridge_k8_d8", 2, 2, OPEN_TIER_PASS, X,
                       status, m);
}

OPEN_GROUP(g_k8_primal) {
  return launch_variant<8, 8, false, cfg(4, 16, 4), cfg(4, 8, 2)>(choice, "ridge_k8_primal", 9, 15, OPEN_TIER_PASS, X,
                       status, m);
}

}  // namespace openk
