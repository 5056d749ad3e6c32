// Ridge-solve kernels of size-class groups, each with its compiled configurations
// (lanes per system, waves per block, waves per SIMD); variant 0 is the default.
#include "rowsolve.h"

namespace openk {

OPEN_GROUP(g_k32_d4) {
  return launch_variant<32, 4, true, cfg(1, 16, 4), cfg(4, 16, 4)>(choice, "ridge_k32_d4", 0, 1, OPEN_TIER_PASS, X,
                       status, m);
}

}  // namespace openk
