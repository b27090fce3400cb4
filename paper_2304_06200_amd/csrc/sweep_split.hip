// Split-column sweep kernels, codes 1 and 3 (see sweep_split.h).
#include "sweep_split.h"

namespace hg {

hipError_t run_split(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  if (sh.ereal) return run_split_e(a, sh, st, ev);
  return sh.pure >= 3 ? split_detail::run_split_code<3>(a, sh, st, ev)
                      : split_detail::run_split_code<1>(a, sh, st, ev);
}

}  // namespace hg
