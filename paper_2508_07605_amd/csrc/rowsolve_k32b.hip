// Ridge-solve kernels of one group of size classes, in their own translation unit.
#include "rowsolve.h"

namespace openk {

open_status classes_k32_mid(OPEN_TIER_ARGS) {
  open_status st;
  if ((st = launch_class<32, 2, 20, true>("ridge_k32_d20", OPEN_TIER_PASS, 5, 5, X, status, m))) return st;
  if ((st = launch_class<32, 2, 24, true>("ridge_k32_d24", OPEN_TIER_PASS, 6, 6, X, status, m))) return st;
  return OPEN_OK;
}

}  // namespace openk
