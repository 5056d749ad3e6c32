// Ridge-solve kernels of one group of size classes, in their own translation unit.
#include "rowsolve.h"

namespace openk {

open_status classes_k32_primal(OPEN_TIER_ARGS) {
  open_status st;
  if ((st = launch_class<32, 4, 32, false>("ridge_k32_primal", OPEN_TIER_PASS, 9, 15, X, status, m))) return st;
  return OPEN_OK;
}

}  // namespace openk
