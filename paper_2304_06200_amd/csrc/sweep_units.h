// Per-width translation units of the sweep kernels (sweep_w*.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "hg_internal.h"
#include "sweep_kernels.h"

namespace hg {

// Per union width W, for PU = 1 (only the main diagonal purely imaginary in B)
// and PU = 3 (it and two more), each with and without the rotated frame of the
// auxiliary vectors (suffix e): one translation unit each.
#define HG_DECLARE_WIDTH(W)                                                                     \
  hipError_t run_width_##W##_p1(const SweepArgs& a, const SweepShape& sh, hipStream_t st,     \
                                hipEvent_t* ev);                                               \
  hipError_t run_width_##W##_p3(const SweepArgs& a, const SweepShape& sh, hipStream_t st,     \
                                hipEvent_t* ev);                                               \
  hipError_t run_width_##W##_p1e(const SweepArgs& a, const SweepShape& sh, hipStream_t st,    \
                                 hipEvent_t* ev);                                              \
  hipError_t run_width_##W##_p3e(const SweepArgs& a, const SweepShape& sh, hipStream_t st,    \
                                 hipEvent_t* ev);
HG_DECLARE_WIDTH(3)
HG_DECLARE_WIDTH(5)
HG_DECLARE_WIDTH(9)
HG_DECLARE_WIDTH(13)
#undef HG_DECLARE_WIDTH
// Row-indexed storage (code bit 3), slot widths 9 and 13, with and without
// the rotated auxiliary frame.
hipError_t run_width_ell_9(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev);
hipError_t run_width_ell_13(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev);

hipError_t launch_integrated(const SweepArgs& a, int nb, hipStream_t st);

// Split-column sweep kernels (sweep_split.hip): 512 threads, 4 rows each,
// union width template 5 or 9, controls of at most 2 diagonals.
hipError_t run_split(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev);
// Zero n counters on the stream (a kernel, so that graph capture records no memset).
hipError_t launch_fill_u32(uint32_t* p, int n, hipStream_t st);

template <typename R, int RPT, int W, int PU, int WK, int G>
hipError_t run_sweep_kernels(const SweepArgs& a, const SweepShape& sh, hipStream_t st,
                             hipEvent_t* ev) {
  auto fk = hg_forward<R, RPT, W, PU, kMaxThreads, false>;
  auto bk = hg_backward<R, RPT, W, PU, WK, G, kMaxThreads, false>;
  if constexpr (W <= 9 && RPT <= (W <= 5 ? 6 : 4)) {
    if (sh.fwd_threads > kMaxThreads) {
      if (sh.fwd_rows_per_thread == 1) fk = hg_forward<R, 1, W, PU, kWideThreads, false>;
      else if (sh.fwd_rows_per_thread == 2) fk = hg_forward<R, 2, W, PU, kWideThreads, false>;
      else if constexpr (W <= 5) fk = hg_forward<R, 3, W, PU, kWideThreads, false>;
      // two state columns per workgroup (complex64, 1-2 rows per thread)
      if constexpr (sizeof(R) == 4 && (PU & 8) == 0) {
        if (sh.fwd_cpw == 2) {
          if (sh.fwd_rows_per_thread == 1) fk = hg_forward<R, 1, W, PU, kWideThreads, false, 2>;
          else fk = hg_forward<R, 2, W, PU, kWideThreads, false, 2>;
        }
      }
    }
  }
  if constexpr (WK <= 2 && ((sizeof(R) == 4 && (RPT <= 2 || (RPT == 3 && W <= 5 && G <= 2))) ||
                             (sizeof(R) == 8 && RPT == 1))) {
    if (sh.threads > kMaxThreads) bk = hg_backward<R, RPT, W, PU, WK, G, kWideThreads, false>;
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fk),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_fwd);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(bk),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bwd);
  if (e != hipSuccess) return e;
  const dim3 grid(sh.n_states, sh.n_batch), block(sh.threads), fblock(sh.fwd_threads);
  const dim3 fgrid(sh.n_states / (sh.fwd_cpw > 1 ? sh.fwd_cpw : 1), sh.n_batch);
  if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
  hipLaunchKernelGGL(fk, fgrid, fblock, sh.lds_fwd, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.ovt && (e = launch_integrated(a, sh.n_batch, st)) != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
  const dim3 bgrid(sh.n_states, sh.n_batch, sh.spread > 1 ? sh.spread : 1);
  hipLaunchKernelGGL(bk, bgrid, block, sh.lds_bwd, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev) e = hipEventRecord(ev[2], st);
  return e;
}

// Dispatch on precision, rows per thread, control width and group size for a
// fixed union width W and kernel code PU (count of purely imaginary leading
// diagonals, plus 4 for the rotated frame of the auxiliary vectors, plus 8 for
// row-indexed storage; both are only built for controls of at most 2 entries
// per row).  complex128 runs at most 6
// rows per thread in one workgroup (its two-vector block leaves LDS above
// about 2400 rows; longer columns are split).
template <int W, int PU>
hipError_t run_width(const SweepArgs& a, const SweepShape& sh, hipStream_t st, hipEvent_t* ev) {
  int wk = 1;
  for (int k = 0; k < a.K; ++k) wk = a.WK[k] > wk ? a.WK[k] : wk;
  constexpr bool ER = (PU & 12) != 0;  // only controls of at most 2 entries per row
#define HG_RUN(R, RPT, WKT, G) return run_sweep_kernels<R, RPT, W, PU, WKT, G>(a, sh, st, ev)
#define HG_BY_G_C64(RPT, WKT)           \
  switch (sh.groups) {                  \
    case 1: HG_RUN(float, RPT, WKT, 1); \
    case 2: HG_RUN(float, RPT, WKT, 2); \
    default: HG_RUN(float, RPT, WKT, 3); \
  }
#define HG_BY_WK(RPT)                                   \
  if (sh.c128) {                                        \
    if constexpr (RPT <= 6) {                           \
      if (ER || wk <= 2) HG_RUN(double, RPT, 2, 1);     \
      if constexpr (!ER) HG_RUN(double, RPT, 4, 1);     \
    }                                                   \
    return hipErrorNotSupported;                        \
  }                                                     \
  if (ER || wk <= 2) { HG_BY_G_C64(RPT, 2) }            \
  if constexpr (!ER) { HG_BY_G_C64(RPT, 4) }            \
  return hipErrorNotSupported;
  switch (sh.rows_per_thread) {
    case 1: { HG_BY_WK(1) }
    case 2: { HG_BY_WK(2) }
    case 3: { HG_BY_WK(3) }
    case 4: { HG_BY_WK(4) }
    case 6: { HG_BY_WK(6) }
    default: { HG_BY_WK(8) }
  }
#undef HG_BY_WK
#undef HG_BY_G_C64
#undef HG_RUN
}

}  // namespace hg
