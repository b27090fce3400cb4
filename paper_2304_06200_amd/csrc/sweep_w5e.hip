// Sweep kernels instantiated for union width 5, the main diagonal purely imaginary in B, auxiliary vectors in the frame of real E_k.
#include "sweep_units.h"

namespace hg {
hipError_t run_width_5_p1e(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  return run_width<5, 5>(a, sh, st, ev);
}
}  // namespace hg
