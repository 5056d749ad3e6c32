// Ridge-solve kernels of one group of size classes, in their own translation unit.
#include "rowsolve.h"

namespace openk {

open_status classes_k64_large(OPEN_TIER_ARGS) {
  open_status st;
  if ((st = launch_class<64, 4, 28, true>("ridge_k64_d28", OPEN_TIER_PASS, 7, 7, X, status, m))) return st;
  if ((st = launch_class<64, 4, 32, true>("ridge_k64_d32", OPEN_TIER_PASS, 8, 8, X, status, m))) return st;
  return OPEN_OK;
}

}  // namespace openk
