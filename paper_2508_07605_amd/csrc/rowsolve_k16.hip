// Ridge-solve kernels of size-class groups, each with its compiled configurations
// (lanes per system, waves per block, waves per SIMD); variant 0 is the default.
#include "rowsolve.h"

namespace openk {

OPEN_GROUP(g_k16_d4) {
  return launch_variant<16, 4, true, cfg(1, 16, 4), cfg(4, 16, 4)>(choice, "ridge_k16_d4", 0, 1, OPEN_TIER_PASS, X,
                       status, m);
}

OPEN_GROUP(g_k16_d8) {
  return launch_variant<16, 8, true, cfg(1, 12, 3), cfg(4, 16, 4)>(choice, "ridge_k16_d8", 2, 2, OPEN_TIER_PASS, X,
                       status, m);
}

OPEN_GROUP(g_k16_d12) {
  return launch_variant<16, 12, true, cfg(1, 8, 2), cfg(4, 16, 4)>(choice, "ridge_k16_d12", 3, 3, OPEN_TIER_PASS, X,
                       status, m);
}

OPEN_GROUP(g_k16_d16) {
  return launch_variant<16, 16, true, cfg(4, 16, 4), cfg(1, 4, 1)>(choice, "ridge_k16_d16", 4, 4, OPEN_TIER_PASS, X,
                       status, m);
}

OPEN_GROUP(g_k16_primal) {
  return launch_variant<16, 16, false, cfg(4, 16, 4), cfg(4, 8, 2)>(choice, "ridge_k16_primal", 9, 15, OPEN_TIER_PASS, X,
                       status, m);
}

}  // namespace openk
