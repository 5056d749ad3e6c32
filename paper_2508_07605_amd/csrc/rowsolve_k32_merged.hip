// The rank-32 ridge solves in three launches instead of one per size class: the primal class
// and the two largest dual classes; the dual classes of 13 to 24 unknowns; the dual classes of
// up to 12 unknowns.  Each launch takes its classes costliest first.  The larger classes run
// four lanes per system, 8 waves per block, 2 per SIMD; the small ones 16 waves per block, 4
// per SIMD (the shapes the autotuner picks for these classes on their own).  The primal and
// largest dual classes stay apart from the middle ones: together they would make the middle
// classes' code spill registers.
#include "rowsolve.h"

namespace openk {

open_status rowsolve_k32_merged(OPEN_TIER_ARGS) {
  open_status st = launch_multi<32, 4, 8, 2, SizeClass<32, false, 9, 15>, SizeClass<32, true, 8, 8>,
                                SizeClass<28, true, 7, 7>>("ridge_k32_d28_up", OPEN_TIER_PASS, X, status, m);
  if (st) return st;
  st = launch_multi<32, 4, 8, 2, SizeClass<24, true, 6, 6>, SizeClass<20, true, 5, 5>, SizeClass<16, true, 4, 4>>(
      "ridge_k32_d16_d24", OPEN_TIER_PASS, X, status, m);
  if (st) return st;
  return launch_multi<32, 4, 16, 4, SizeClass<12, true, 3, 3>, SizeClass<8, true, 2, 2>, SizeClass<4, true, 0, 1>>(
      "ridge_k32_d4_d12", OPEN_TIER_PASS, X, status, m);
}

}  // namespace openk
