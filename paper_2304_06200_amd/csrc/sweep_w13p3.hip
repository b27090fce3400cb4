// Sweep kernels instantiated for union width 13, three leading diagonals purely imaginary in B.
#include "sweep_units.h"

namespace hg {
hipError_t run_width_13_p3(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  return run_width<13, 3>(a, sh, st, ev);
}
}  // namespace hg
