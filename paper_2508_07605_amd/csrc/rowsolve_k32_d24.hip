// Ridge-solve kernels of size-class groups, each with its compiled configurations
// (lanes per system, waves per block, waves per SIMD); variant 0 is the default.
#include "rowsolve.h"

namespace openk {

OPEN_GROUP(g_k32_d24) {
  return launch_variant<32, 24, true, cfg(4, 12, 3), cfg(4, 8, 2), cfg(2, 4, 1), cfg(4, 8, 2, 1)>(choice, "ridge_k32_d24", 6, 6, OPEN_TIER_PASS, X,
                       status, m);
}

}  // namespace openk
