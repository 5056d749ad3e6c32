// Ridge-solve kernels of one group of size classes, in their own translation unit.
#include "rowsolve.h"

namespace openk {

open_status classes_k8(OPEN_TIER_ARGS) {
  open_status st;
  if ((st = launch_class<8, 1, 4, true>("ridge_k8_d4", OPEN_TIER_PASS, 0, 1, X, status, m))) return st;
  if ((st = launch_class<8, 1, 8, true>("ridge_k8_d8", OPEN_TIER_PASS, 2, 2, X, status, m))) return st;
  if ((st = launch_class<8, 4, 8, false>("ridge_k8_primal", OPEN_TIER_PASS, 9, 15, X, status, m))) return st;
  return OPEN_OK;
}

}  // namespace openk
