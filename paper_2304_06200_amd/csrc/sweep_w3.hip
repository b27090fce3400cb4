// Sweep kernels instantiated for union width 3, the main diagonal purely imaginary in B.
#include "sweep_units.h"

namespace hg {
hipError_t run_width_3_p1(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  return run_width<3, 1>(a, sh, st, ev);
}
}  // namespace hg
