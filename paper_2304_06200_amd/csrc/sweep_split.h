// Split-column sweep kernels: a state column too long for one workgroup runs
// as P co-resident workgroups (see Split in hg_internal.h) that exchange their
// edge rows after every Taylor term.  Instantiated for 512 threads with 4 rows
// each (up to 2048 local rows), union width templates 5 and 9 and controls of
// at most 2 diagonals; launched cooperatively so that the runtime places all
// workgroups of the grid at once (the parts of a column wait on each other).
// Kernel codes as for the single-workgroup kernels (sweep_units.h): 1 or 3
// purely imaginary leading diagonals, +4 for the rotated auxiliary frame;
// codes 1 and 3 are built in sweep_split.hip, 5 and 7 in sweep_split_e.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "hg_internal.h"
#include "sweep_kernels.h"
#include "sweep_units.h"

namespace hg {
namespace split_detail {

template <typename R, int W, int PU, int G>
hipError_t run_split_kernels(const SweepArgs& a0, const SweepShape& sh, hipStream_t st,
                             hipEvent_t* ev) {
  auto fk = hg_forward<R, 4, W, PU, kMaxThreads, true>;
  auto bk = hg_backward<R, 4, W, PU, 2, G, kMaxThreads, true>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fk),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_fwd);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(bk),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bwd);
  if (e != hipSuccess) return e;
  SweepArgs a = a0;
  void* args[] = {&a};
  const dim3 grid(sh.n_states, sh.n_batch), block(kMaxThreads);
  const int nflags = sh.n_states * sh.n_batch;
  if ((e = launch_fill_u32(a.xflag, nflags, st)) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fk), grid, block, args,
                                 (unsigned)sh.lds_fwd, st);
  if (e != hipSuccess) return e;
  if (a.ovt && (e = launch_integrated(a, sh.n_batch, st)) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.xflag, nflags, st)) != hipSuccess) return e;
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(bk), grid, block, args,
                                 (unsigned)sh.lds_bwd, st);
  if (e != hipSuccess) return e;
  if (ev) e = hipEventRecord(ev[2], st);
  return e;
}

template <int W, int PU>
hipError_t run_split_width(const SweepArgs& a, const SweepShape& sh, hipStream_t st,
                           hipEvent_t* ev) {
  if (sh.c128) return run_split_kernels<double, W, PU, 1>(a, sh, st, ev);
  switch (sh.groups) {
    case 1: return run_split_kernels<float, W, PU, 1>(a, sh, st, ev);
    case 2: return run_split_kernels<float, W, PU, 2>(a, sh, st, ev);
    default: return run_split_kernels<float, W, PU, 3>(a, sh, st, ev);
  }
}


template <int PU>
hipError_t run_split_code(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  if (a.W <= 5) return run_split_width<5, PU>(a, sh, st, ev);
  return run_split_width<9, PU>(a, sh, st, ev);
}

}  // namespace split_detail

// codes 5 and 7 (sweep_split_e.hip)
hipError_t run_split_e(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev);

}  // namespace hg
