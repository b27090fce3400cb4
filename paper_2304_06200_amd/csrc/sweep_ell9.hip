// Sweep kernels for row-indexed storage with 9 slots per row (the main
// diagonal purely imaginary in B), with and without the rotated auxiliary frame.
#include "sweep_units.h"

namespace hg {
hipError_t run_width_ell_9(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  if (sh.ereal) return run_width<9, 13>(a, sh, st, ev);
  return run_width<9, 9>(a, sh, st, ev);
}
}  // namespace hg
