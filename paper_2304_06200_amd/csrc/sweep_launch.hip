// Launchers: step norms (App. C 1-norm), state norms, the sweep kernels and
// the deterministic gradient reduction.  Kernel templates are instantiated
// here for the supported (precision, rows per thread, union width, control
// width) combinations; wider problems are rejected with HG_ERR_UNSUPPORTED.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>

#include "hg_internal.h"
#include "sweep_kernels.h"
#include "sweep_units.h"

namespace hg {

// theta[b][n] = dt * max_i sum_j |(H_0 + sum_k u[b][k][n] H_k)_ij| in FP64.
// Row sums equal column sums because H_n is Hermitian (App. C, eq. norm
// inequality and its footnote).  A non-finite amplitude yields a NaN norm.
__global__ void __launch_bounds__(256) k_step_norms(const double2* vals, int W, int d, int K,
                                                    const double* u, int N, double dt,
                                                    double* theta) {
  __shared__ double red[4];
  const int n = blockIdx.x, b = blockIdx.y;
  const double* ub = u + (size_t)b * K * N;
  double mx = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    double rs = 0.0;
    for (int e = 0; e < W; ++e) {
      const double2 v0 = vals[(size_t)e * d + i];
      double hr = v0.x, hi = v0.y;
      for (int k = 0; k < K; ++k) {
        const double c = ub[(size_t)k * N + n];
        const double2 v = vals[((size_t)(k + 1) * W + e) * d + i];
        hr = fma(c, v.x, hr);
        hi = fma(c, v.y, hi);
      }
      rs += hypot(hr, hi);
    }
    mx = (rs > mx || rs != rs) ? rs : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double t = __shfl_xor(mx, o, 64);
    mx = (t > mx || t != t) ? t : mx;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = (red[w] > r || red[w] != red[w]) ? red[w] : r;
    theta[(size_t)b * N + n] = dt * r;
  }
}

// ||psi^h|| for every state of every batch entry (FP64).
__global__ void __launch_bounds__(256) k_state_norms(const double2* psi, int d, int S,
                                                     double* out) {
  __shared__ double red[4];
  const int h = blockIdx.x, b = blockIdx.y;
  const double2* p = psi + ((size_t)b * S + h) * d;
  double s = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) s += p[i].x * p[i].x + p[i].y * p[i].y;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    out[(size_t)b * S + h] = sqrt(t);
  }
}

// grad[b][k][n] = sum_h gradp[b][h][k][n], h ascending (deterministic).
__global__ void __launch_bounds__(256) k_reduce_grad(const double* gradp, double* grad, int S,
                                                     int KN, int B) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * KN) return;
  const size_t b = idx / KN, kn = idx % KN;
  double s = 0.0;
  for (int h = 0; h < S; ++h) s += gradp[(b * S + h) * KN + kn];
  grad[idx] = s;
}

// Time-integrated infidelity (App. A): g_n = (1/S) sum_h <phi_T^h|psi_n^h> for
// every step (h ascending) and C3 = 1 - (1/N) sum_n |g_n|^2 per evaluation
// (fixed-order block reduction), written to res[b][5].  One block per b.
__global__ void __launch_bounds__(256) k_integrated(const double* ovt, double* gt, double* res,
                                                    int S, int St, int N) {
  __shared__ double red[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  double acc = 0.0;
  for (int n = tid; n < N; n += 256) {
    double gr = 0.0, gi = 0.0;
    for (int h = 0; h < S; ++h) {
      gr += ovt[(((size_t)b * S + h) * N + n) * 2 + 0];
      gi += ovt[(((size_t)b * S + h) * N + n) * 2 + 1];
    }
    gr /= St;  // S local columns (a split column has several) of St states
    gi /= St;
    gt[((size_t)b * N + n) * 2 + 0] = gr;
    gt[((size_t)b * N + n) * 2 + 1] = gi;
    acc += gr * gr + gi * gi;
  }
  red[tid] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) res[(size_t)b * 8 + 5] = 1.0 - red[0] / N;
}

hipError_t launch_integrated(const SweepArgs& a, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_integrated, dim3(nb), dim3(256), 0, st, a.ovt, a.gt, a.res, a.S, a.St, a.N);
  return hipGetLastError();
}

hipError_t launch_step_norms(const DevOps& ops, int dim, int K, const double* u, int nb, int N,
                             double dt, double* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_step_norms, dim3(N, nb), dim3(256), 0, st, ops.vals, ops.W, dim, K, u, N,
                     dt, theta);
  return hipGetLastError();
}

hipError_t launch_state_norms(const double* psi, int dim, int S, int nb, double* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_state_norms, dim3(S, nb), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(psi), dim, S, out);
  return hipGetLastError();
}

namespace {

constexpr int kWidths[] = {3, 5, 9, 13};

int width_template(int W) {
  for (int w : kWidths)
    if (W <= w) return w;
  return -1;
}

size_t lds_bytes(int vecs, int rpt, int dim, int halo, size_t csize) {
  return (size_t)kRedBytes + (size_t)block_bytes((int)csize, rpt, vecs, dim, halo);
}

}  // namespace

bool sweep_supported(const DevOps& ops, int dim, int K, bool c128, size_t lds_limit,
                     SweepShape* sh, std::string* why) {
  if (K > kMaxCtrl) {
    *why = "more than " + std::to_string(kMaxCtrl) + " controls";
    return false;
  }
  int rpt = (dim + kMaxThreads - 1) / kMaxThreads;
  rpt = rpt <= 4 ? rpt : rpt <= 6 ? 6 : 8;
  if (rpt > kMaxRows) {
    *why = "dimension " + std::to_string(dim) + " exceeds " +
           std::to_string(kMaxRows * kMaxThreads) + " (rows per thread)";
    return false;
  }
  if (width_template(ops.W) < 0) {
    *why = "union pattern has " + std::to_string(ops.W) + " diagonals (max 13)";
    return false;
  }
  // one row per thread below 512 rows; above, 8 full waves (2 per SIMD) and
  // the kernels skip wave slabs past the dimension, which balances the SIMDs
  int threads = rpt == 1 ? ((dim + 63) / 64) * 64 : kMaxThreads;
  const size_t cs = c128 ? 16 : 8;
  // Above 512 rows (up to 2048): 1024 threads (4 waves per SIMD, to hide the
  // latency around each term's barrier) with 1 or 2 rows each; the LDS layout
  // is that of 2*rows per 512 threads.  The forward always, the backward in
  // complex64 when its controls have at most 2 diagonals (register budget).
  int wk = 1;
  for (int k = 0; k < K; ++k) wk = std::max(wk, ops.WK[k]);
  int frpt = rpt, fthreads = threads, flr = rpt, blr = rpt;
  // (not for row-indexed storage, whose gather columns take registers)
  const bool wide = !ops.ell && dim > kMaxThreads && ((dim <= 2 * kWideThreads && ops.W <= 9) ||
                                          (dim <= 3 * kWideThreads && ops.W <= 5));
  if (wide) {
    frpt = (dim + kWideThreads - 1) / kWideThreads;
    fthreads = frpt == 1 ? ((dim + 63) / 64) * 64 : kWideThreads;
    flr = frpt * kWideThreads / kMaxThreads;
    // the backward too: complex64 with controls of at most 2 diagonals, and
    // complex128 at one row per thread (up to 1024 rows)
    if (wk <= 2 && (!c128 || frpt == 1)) {
      rpt = frpt;
      threads = fthreads;
      blr = flr;
    }
  }
  const size_t fwd = lds_bytes(1, flr, dim, ops.halo, cs);
  if (fwd > lds_limit) {
    *why = "forward term vectors need " + std::to_string(fwd) + " B of LDS";
    return false;
  }
  // controls per backward pass: complex128 keeps one (register budget); complex64
  // prefers a group size that divides K so no pass carries idle vectors
  int G = 1;
  if (!c128 && K >= 2) G = (K % 3 == 0) ? 3 : (K % 2 == 0) ? 2 : (K >= 3 ? 3 : 2);
  auto bwd_bytes = [&](int g) {
    return std::max(lds_bytes(2, blr, dim, ops.halo, cs), lds_bytes(g + 1, blr, dim, ops.halo, cs));
  };
  // 3 rows per thread at 1024 threads leaves registers for two controls per pass
  if (!c128 && threads > kMaxThreads && rpt == 3 && G > 2) G = 2;
  while (G > 1 && bwd_bytes(G) > lds_limit) --G;
  if (bwd_bytes(G) > lds_limit) {
    *why = "backward state block does not fit in LDS";
    return false;
  }
  sh->dim = dim;
  sh->n_ctrl = K;
  sh->rows_per_thread = rpt;
  sh->threads = threads;
  sh->fwd_rows_per_thread = frpt;
  sh->fwd_threads = fthreads;
  sh->fwd_cpw = 1;
  // two columns per forward workgroup: complex64, 1024 threads, 1-2 rows each
  sh->lds_fwd2 = (!c128 && wide && frpt <= 2) ? lds_bytes(2, flr, dim, ops.halo, cs) : 0;
  sh->groups = G;
  sh->lds_fwd = fwd;
  sh->lds_bwd = bwd_bytes(G);
  sh->c128 = c128;
  return true;
}

hipError_t launch_sweep(const DevOps& ops, const SweepShape& sh, const SweepBuffers& bf,
                        const SweepParams& p, hipStream_t st) {
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.d = sh.dim;
  a.K = sh.n_ctrl;
  a.N = sh.n_steps;
  a.S = sh.n_states;
  a.W = ops.W;
  a.halo = ops.halo;
  a.G = sh.groups;
  a.renorm_every = p.renorm_every;
  a.ckpt_every = p.ckpt_every;
  for (int e = 0; e < kMaxDiag; ++e) a.off[e] = e < ops.W ? ops.off[e] : 0;
  int wk = 1;
  for (int k = 0; k < kMaxCtrl; ++k) {
    a.WK[k] = k < sh.n_ctrl ? ops.WK[k] : 0;
    if (k < sh.n_ctrl && ops.WK[k] > wk) wk = ops.WK[k];
    for (int q = 0; q < kMaxDiagCtrl; ++q) a.offk[k][q] = (k < sh.n_ctrl && q < ops.WK[k]) ? ops.offk[k][q] : 0;
    a.ecl[k] = k < sh.n_ctrl ? ops.ecl[k] : 0;
  }
  a.vals = ops.vals;
  a.valk = ops.valk;
  a.cols = ops.ell ? ops.cols : nullptr;
  a.colk = ops.ell ? ops.colk : nullptr;
  a.omega = ops.omega;
  a.u = bf.u;
  a.msch = bf.m_sched;
  a.ssch = bf.s_sched;
  a.psi0 = reinterpret_cast<const double2*>(bf.psi0);
  a.tgt = reinterpret_cast<const double2*>(bf.targets);
  a.psiN = bf.psiN;
  a.cold = bf.cold;
  a.ckpt = bf.ckpt;
  a.segbuf = bf.segbuf;
  a.ovl = bf.ovl;
  a.ovt = bf.ovt;
  a.gt = bf.gt;
  a.pen = bf.pen;
  a.gradp = bf.gradp;
  a.drift = bf.drift;
  a.res = bf.res;
  a.dt = p.dt;
  a.w_fid = p.w_fid;
  a.w_pen = p.w_pen;
  a.w_int = p.w_int;
  a.P = 1;
  a.St = sh.n_states;
  hipError_t e;
  hipEvent_t* ev = bf.ev[0] ? const_cast<hipEvent_t*>(bf.ev) : nullptr;
  const int code = (sh.pure >= 3 ? 1 : 0) + (sh.ereal ? 2 : 0);
#define HG_BY_CODE(W)                                    \
  switch (code) {                                        \
    case 0: e = run_width_##W##_p1(a, sh, st, ev); break;  \
    case 1: e = run_width_##W##_p3(a, sh, st, ev); break;  \
    case 2: e = run_width_##W##_p1e(a, sh, st, ev); break; \
    default: e = run_width_##W##_p3e(a, sh, st, ev); break; \
  }
  if (ops.ell) {  // row-indexed storage: slot widths 9 and 13
    e = ops.W <= 9 ? run_width_ell_9(a, sh, st, ev) : run_width_ell_13(a, sh, st, ev);
  } else {
    switch (width_template(ops.W)) {
      case 3: HG_BY_CODE(3) break;
      case 5: HG_BY_CODE(5) break;
      case 9: HG_BY_CODE(9) break;
      default: HG_BY_CODE(13) break;
    }
  }
#undef HG_BY_CODE
  if (e != hipSuccess) return e;
  if (bf.grad && sh.n_ctrl > 0) {
    const size_t total = (size_t)sh.n_batch * sh.n_ctrl * sh.n_steps;
    hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       bf.gradp, bf.grad, sh.n_states, sh.n_ctrl * sh.n_steps, sh.n_batch);
    e = hipGetLastError();
  }
  return e;
}

// ------------------------------------------------------------ split columns --
namespace {

struct SplitLayout {
  int P, L, T, h, seg, d_loc;
  int w[kMaxParts], c0[kMaxParts];
};

// dst[b][h*P + q][l] = src[b][h][global row of local row l of part q], zero on
// halo and padding rows.
__global__ void __launch_bounds__(256) k_split_gather(const double2* __restrict__ src,
                                                      double2* __restrict__ dst, int d, int St,
                                                      SplitLayout sl) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= sl.d_loc) return;
  const int hp = blockIdx.y, b = blockIdx.z;
  const int h = hp / sl.P, q = hp % sl.P;
  const int t = l / sl.seg, k = l % sl.seg - sl.h;
  double2 v = {0.0, 0.0};
  if (k >= 0 && k < sl.w[q]) v = src[((size_t)b * St + h) * d + (size_t)t * sl.L + sl.c0[q] + k];
  dst[((size_t)b * St * sl.P + hp) * sl.d_loc + l] = v;
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

bool split_supported(const Split& sp, int K, bool c128, size_t lds_limit, int num_cu,
                     SweepShape* sh, std::string* why) {
  (void)num_cu;
  if (sp.P < 2) {
    *why = "no split";
    return false;
  }
  if (K > kMaxCtrl) {
    *why = "more than " + std::to_string(kMaxCtrl) + " controls";
    return false;
  }
  if (sp.d_loc > 4 * kMaxThreads) {
    *why = "a part of " + std::to_string(sp.d_loc) + " local rows exceeds the split kernels' " +
           std::to_string(4 * kMaxThreads);
    return false;
  }
  if (sp.ops.W > 9) {
    *why = "the split kernels take at most 9 union diagonals";
    return false;
  }
  for (int k = 0; k < K; ++k)
    if (sp.ops.WK[k] > 2) {
      *why = "the split kernels take controls of at most 2 diagonals";
      return false;
    }
  const size_t cs = c128 ? 16 : 8;
  const size_t fwd = lds_bytes(1, 4, sp.d_loc, sp.ops.halo, cs);
  auto bwd_bytes = [&](int g) {
    return std::max(lds_bytes(2, 4, sp.d_loc, sp.ops.halo, cs),
                    lds_bytes(g + 1, 4, sp.d_loc, sp.ops.halo, cs));
  };
  int G = 1;
  if (!c128 && K >= 2) G = (K % 3 == 0) ? 3 : (K % 2 == 0) ? 2 : (K >= 3 ? 3 : 2);
  while (G > 1 && bwd_bytes(G) > lds_limit) --G;
  if (fwd > lds_limit || bwd_bytes(G) > lds_limit) {
    *why = "a part's term vectors do not fit in LDS";
    return false;
  }
  sh->dim = sp.d_loc;
  sh->n_ctrl = K;
  sh->rows_per_thread = 4;
  sh->threads = kMaxThreads;
  sh->fwd_rows_per_thread = 4;
  sh->fwd_threads = kMaxThreads;
  sh->groups = G;
  sh->lds_fwd = fwd;
  sh->lds_bwd = bwd_bytes(G);
  sh->c128 = c128;
  sh->parts = sp.P;
  return true;
}

hipError_t launch_split_sweep(const Split& sp, const SweepShape& sh0, const SweepBuffers& bf,
                              const SplitBuffers& x, const SweepParams& p, int S_true,
                              hipStream_t st) {
  const int P = sp.P, B = sh0.n_batch, Sl = S_true * P;
  SplitLayout sl{};
  sl.P = P;
  sl.L = sp.L;
  sl.T = sp.T;
  sl.h = sp.h;
  sl.seg = sp.seg;
  sl.d_loc = sp.d_loc;
  for (int q = 0; q < kMaxParts; ++q) {
    sl.w[q] = sp.w[q];
    sl.c0[q] = sp.c0[q];
  }
  const int dim = sp.L * sp.T;
  const dim3 gg((sp.d_loc + 255) / 256, Sl, B);
  hipLaunchKernelGGL(k_split_gather, gg, dim3(256), 0, st,
                     reinterpret_cast<const double2*>(bf.psi0), x.psi0_loc, dim, S_true, sl);
  hipLaunchKernelGGL(k_split_gather, gg, dim3(256), 0, st,
                     reinterpret_cast<const double2*>(bf.targets), x.tgt_loc, dim, S_true, sl);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, x.xerr, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  SweepShape sh = sh0;
  sh.n_states = Sl;
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  const DevOps& ops = sp.ops;
  a.d = sp.d_loc;
  a.K = sh.n_ctrl;
  a.N = sh.n_steps;
  a.S = Sl;
  a.W = ops.W;
  a.halo = ops.halo;
  a.G = sh.groups;
  a.renorm_every = p.renorm_every;
  a.ckpt_every = p.ckpt_every;
  for (int q = 0; q < kMaxDiag; ++q) a.off[q] = q < ops.W ? ops.off[q] : 0;
  for (int k = 0; k < kMaxCtrl; ++k) {
    a.WK[k] = k < sh.n_ctrl ? ops.WK[k] : 0;
    for (int q = 0; q < kMaxDiagCtrl; ++q)
      a.offk[k][q] = (k < sh.n_ctrl && q < ops.WK[k]) ? ops.offk[k][q] : 0;
    a.ecl[k] = k < sh.n_ctrl ? ops.ecl[k] : 0;
  }
  a.vals = ops.vals;
  a.valk = ops.valk;
  a.cols = ops.ell ? ops.cols : nullptr;
  a.colk = ops.ell ? ops.colk : nullptr;
  a.omega = ops.omega;
  a.u = bf.u;
  a.msch = bf.m_sched;
  a.ssch = bf.s_sched;
  a.psi0 = x.psi0_loc;
  a.tgt = x.tgt_loc;
  a.psiN = bf.psiN;
  a.cold = bf.cold;
  a.ckpt = bf.ckpt;
  a.segbuf = bf.segbuf;
  a.ovl = bf.ovl;
  a.ovt = bf.ovt;
  a.gt = bf.gt;
  a.pen = bf.pen;
  a.gradp = bf.gradp;
  a.drift = bf.drift;
  a.res = bf.res;
  a.dt = p.dt;
  a.w_fid = p.w_fid;
  a.w_pen = p.w_pen;
  a.w_int = p.w_int;
  a.P = P;
  a.St = S_true;
  a.xT = sp.T;
  a.xh = sp.h;
  a.xseg = sp.seg;
  a.xrows = sp.T * std::max(sp.h, 1);
  for (int q = 0; q < kMaxParts; ++q) a.xw[q] = sp.w[q];
  a.psv = sp.vals_stride;
  a.psk = sp.valk_stride;
  a.pso = sp.omega_stride;
  a.xbuf = x.xbuf;
  a.xnrm = x.xnrm;
  a.xflag = x.xflag;
  a.xerr = x.xerr;
  // longest wait for a neighbour; HG_SPLIT_WAIT_TICKS (100 MHz ticks) shortens
  // it, which lets a test drive the timeout path with every kernel exiting normally
  a.xwait = kXWaitTicks;
  if (const char* env = std::getenv("HG_SPLIT_WAIT_TICKS")) {
    char* end = nullptr;
    const unsigned long long v = std::strtoull(env, &end, 10);
    if (end && end != env) a.xwait = v;
  }
  e = run_split(a, sh, st, bf.ev[0] ? const_cast<hipEvent_t*>(bf.ev) : nullptr);
  if (e != hipSuccess) return e;
  if (bf.grad && sh.n_ctrl > 0) {
    const size_t total = (size_t)B * sh.n_ctrl * sh.n_steps;
    hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       bf.gradp, bf.grad, Sl, sh.n_ctrl * sh.n_steps, B);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_fill_u32(uint32_t* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace hg
