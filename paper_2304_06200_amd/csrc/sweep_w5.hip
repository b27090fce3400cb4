// Sweep kernels instantiated for union width 5, the main diagonal purely imaginary in B.
#include "sweep_units.h"

namespace hg {
hipError_t run_width_5_p1(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  return run_width<5, 1>(a, sh, st, ev);
}
}  // namespace hg
