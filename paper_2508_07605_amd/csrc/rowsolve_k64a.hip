// Ridge-solve kernels of one group of size classes, in their own translation unit.
#include "rowsolve.h"

namespace openk {

open_status classes_k64_small(OPEN_TIER_ARGS) {
  open_status st;
  if ((st = launch_class<64, 1, 4, true>("ridge_k64_d4", OPEN_TIER_PASS, 0, 1, X, status, m))) return st;
  if ((st = launch_class<64, 1, 8, true>("ridge_k64_d8", OPEN_TIER_PASS, 2, 2, X, status, m))) return st;
  if ((st = launch_class<64, 1, 12, true>("ridge_k64_d12", OPEN_TIER_PASS, 3, 3, X, status, m))) return st;
  if ((st = launch_class<64, 1, 16, true>("ridge_k64_d16", OPEN_TIER_PASS, 4, 4, X, status, m))) return st;
  return OPEN_OK;
}

}  // namespace openk
