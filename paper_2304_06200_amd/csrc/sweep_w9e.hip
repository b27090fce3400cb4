// Sweep kernels instantiated for union width 9, the main diagonal purely imaginary in B, auxiliary vectors in the frame of real E_k.
#include "sweep_units.h"

namespace hg {
hipError_t run_width_9_p1e(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  return run_width<9, 5>(a, sh, st, ev);
}
}  // namespace hg
