// Split-column sweep kernels, codes 5 and 7: the auxiliary vectors in the
// frame of real E_k (see sweep_split.h).
#include "sweep_split.h"

namespace hg {

hipError_t run_split_e(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  return sh.pure >= 3 ? split_detail::run_split_code<7>(a, sh, st, ev)
                      : split_detail::run_split_code<5>(a, sh, st, ev);
}

}  // namespace hg
