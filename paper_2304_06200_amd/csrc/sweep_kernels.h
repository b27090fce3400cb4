// Device code of the HG-GRAPE sweep for gfx950 (included by sweep_w*.hip).
//
// Work decomposition.  One workgroup owns one state column h of one
// evaluation b for the whole time axis (the chain psi_0 -> psi_N is strictly
// sequential, Sec. II).  Each thread owns RPT rows (row = tid + r*NT, so a
// wavefront touches consecutive rows); workgroups have 512 threads (2
// wavefronts per SIMD) or, where registers allow, 1024 (4 per SIMD, which
// hides the latency around each term's barrier).  For step n the thread
// assembles its rows of B_n = -i dt H_n / s_n on the W union diagonals into
// registers once and reuses them for all m_n s_n Taylor terms.
//
// Term vectors live in LDS as a *state block*: row i of the block holds the
// V vectors that are propagated together (1 in the forward sweep, psi and
// Lambda in the reconstruction, Y and X_1..X_G in the auxiliary action), so
// one wide ds_read per (row, diagonal) fetches all of them and one address
// register per (row, diagonal) serves every vector.  The block is double
// buffered (one barrier per Taylor term) and framed by `halo` zero rows on
// both sides, so the shifted reads at i + off_e need no clamping or bounds
// tests.  Accumulators stay in registers.  Norms, overlaps and gradient
// partials are accumulated in FP64 and reduced in a fixed order
// (deterministic, bitwise reproducible).
#pragma once

#include <hip/hip_runtime.h>

#include "hg_internal.h"

namespace hg {

constexpr int kRedBytes = 1024;  // FP64 reduction scratch at the start of LDS

template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R re, im;
};

// The vectors a sweep carries from term to term and step to step (psi, and
// Lambda in the backward) accumulate in FP64 in both precisions; only the
// copies that feed the next term's products are rounded to R.
using CA = cx<double>;
template <typename T, typename U>
__device__ __forceinline__ cx<T> cxc(const cx<U>& x) {
  return cx<T>{(T)x.re, (T)x.im};
}
// FP64 sums over the carried vectors are written as explicit FMA chains: the
// compiler may not contract them differently in different kernel variants, so
// a column gives bitwise the same norms and overlaps whichever variant runs it.
__device__ __forceinline__ double acc_norm2(double s, CA z) {
  return fma(z.im, z.im, fma(z.re, z.re, s));
}
// s + conj(t) z
__device__ __forceinline__ void acc_dot(double& sr, double& si, double2 t, CA z) {
  sr = fma(t.y, z.im, fma(t.x, z.re, sr));
  si = fma(-t.y, z.re, fma(t.x, z.im, si));
}

struct SweepArgs {
  int d, K, N, S, W, halo, G, renorm_every;
  int ckpt_every;        // > 0: checkpointed-state variant, psi stored every ckpt_every steps
  int off[kMaxDiag];
  int WK[kMaxCtrl];
  int offk[kMaxCtrl][kMaxDiagCtrl];
  int ecl[kMaxCtrl];  // control classes of a rotated-frame backward (DevOps::ecl)
  const int32_t* cols;  // row-indexed storage: [W][d] columns of the union slots (DevOps::cols)
  const int32_t* colk;  // row-indexed storage: [K][kMaxDiagCtrl][d] control columns
  const double2* vals;   // [(K+1)][W][d]
  const double2* valk;   // [K][kMaxDiagCtrl][d]
  const double* omega;   // [d] or nullptr
  const double* u;       // [B][K][N]
  const int* msch;       // [B][N]
  const int* ssch;       // [B][N]
  const double2* psi0;   // [B][S][d]
  const double2* tgt;    // [B][S][d]
  void* psiN;            // [B][S][d] (working precision)
  void* cold;            // [B][S][Q][3][d] complex FP64 (Q = gridDim.z of the backward)
  void* ckpt;            // [B][S][ceil(N/C)][d] checkpoints psi_0, psi_C, ... (checkpoint variant)
  void* segbuf;          // [B][S][Q][C][d] states of the segment being swept back
  double* ovl;           // [B][S][2]
  double* ovt;           // [B][S][N][2] overlap after each step, or null (no C3 term)
  double* gt;            // [B][N][2] g_n = (1/S) sum_h ovt (filled between the sweeps)
  double* pen;           // [B][S]
  double* gradp;         // [B][S][K][N]
  double* drift;         // [B][S]
  double* res;           // [B][8]
  double dt, w_fid, w_pen, w_int;
  // Split columns (P > 1): local column h = h_true * P + part, S = S_true * P;
  // vals/valk/omega hold P parts back to back (strides psv, psk, pso).
  int P, St;             // parts per column (1: no split), true number of states
  int xT, xh, xseg, xrows;  // blocks, halo rows per side, local rows per block, xT * xh
  int xw[kMaxParts];     // own rows per block of each part
  size_t psv, psk, pso;
  unsigned char* xbuf;   // [B][S][2 slots][2 sides][xrows][kXRowBytes] edge rows
  double* xnrm;          // [B][S][kMaxParts] partial norms (ring of slots)
  uint32_t* xflag;       // [B][S] last exchange each local column has published
  uint32_t* xerr;        // [1] non-zero once a wait timed out
  uint64_t xwait;        // longest wait, ticks of the 100 MHz real-time counter
};

constexpr int kXRowBytes = 64;                   // bytes reserved per exchanged row
constexpr uint64_t kXWaitTicks = 2000000000ull;  // default longest wait: 20 s at 100 MHz

template <typename R>
__device__ __forceinline__ void cmac(cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

// acc += a b for a purely imaginary a (a.re is not read): the two
// multiply-adds of cmac whose factor a.re is zero are left out, which gives
// the same result (up to the sign of a zero).
template <typename R>
__device__ __forceinline__ void cmac_im(cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.im, b.re, acc.im);
}

// Coefficient q of a row of B: the first PU union diagonals are those on which
// every operator is real, where B = -i (dt/s) H is purely imaginary.  The
// kernels' PU template code carries this count in its low two bits (1 or 3)
// and, in bit 2, the rotated frame of the auxiliary vectors (emac).
template <int PU, typename R>
__device__ __forceinline__ void bmac(int q, cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  if (q < (PU & 3))
    cmac_im(acc, a, b);
  else
    cmac(acc, a, b);
}

// acc += E_k y for the top block of an auxiliary vector.  In the rotated frame
// (PU bit 2) the block holds X_k / w_k, whose source e_k y has the real factor
// e_k (load_E): two multiply-adds.  Multiplying by w_k in {1, -i} is exact, so
// only the overlap with the co-state needs to know the frame.
template <int PU, typename R>
__device__ __forceinline__ void emac(cx<R>& acc, const cx<R>& e, const cx<R>& y) {
  if constexpr ((PU & 4) != 0) {
    acc.re = fma(e.re, y.re, acc.re);
    acc.im = fma(e.re, y.im, acc.im);
  } else {
    cmac(acc, e, y);
  }
}

// Hide a value from loop-invariant code motion: address arithmetic built on
// it is redone where it is used instead of being hoisted out of the time loop
// (which would pin one 64-bit address per operator entry in registers).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
// The same for a wave-uniform value kept in a scalar register: the compiler
// then adds it with one scalar op instead of splitting it into vector adds.
__device__ __forceinline__ uint32_t opaque_s(uint32_t x) {
  asm volatile("" : "+s"(x));
  return x;
}

// Whether any row of this wavefront's slab r exists (wave-uniform, kept in a
// scalar register): whole slabs past the dimension are skipped, not masked.
template <int RPT>
__device__ __forceinline__ void slab_valid(int d, bool (&sv)[RPT]) {
  const int w0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
#pragma unroll
  for (int r = 0; r < RPT; ++r) sv[r] = RPT == 1 || w0 + r * (int)blockDim.x < d;
}

// Deterministic FP64 block sum of NV values; every thread receives the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  static_assert(NV * 16 * 8 <= 512, "the reduction scratch ends where the 1/j table starts");
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * 16 + w] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[i * 16 + k];
    v[i] = s;
  }
}

// Rows of B_n = -i (dt/s) (H_0 + sum_k u_k H_k) on the union diagonals,
// assembled in FP64 and rounded once to the working precision.
template <typename R, int RPT, int W>
__device__ __forceinline__ void assemble_B(const SweepArgs& a, const double2* vals,
                                           const double* ub, int n,
                                           const int (&row)[RPT], const bool (&ok)[RPT],
                                           double cs, cx<R> (&bv)[RPT][W]) {
  const int d = a.d;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = opaque(row[r]);
#pragma unroll
    for (int e = 0; e < W; ++e) {
      double hr = 0.0, hi = 0.0;
      if (e < a.W && ok[r]) {
        const double2 v0 = vals[(size_t)e * d + i];
        hr = v0.x;
        hi = v0.y;
        for (int k = 0; k < a.K; ++k) {
          const double c = ub[(size_t)k * a.N + n];
          const double2 v = vals[((size_t)(k + 1) * a.W + e) * d + i];
          hr = fma(c, v.x, hr);
          hi = fma(c, v.y, hi);
        }
      }
      bv[r][e].re = (R)(cs * hi);
      bv[r][e].im = (R)(-cs * hr);
    }
  }
}

// Row-indexed storage (kernel code bit 3): the gather column of union slot q
// for each row of this thread (the row itself where the slot is padding).
template <int RPT, int W, bool ELL>
__device__ __forceinline__ void load_cols(const SweepArgs& a, const int (&row)[RPT], int (&cl)[RPT][W]) {
#pragma unroll
  for (int r = 0; r < RPT; ++r)
#pragma unroll
    for (int q = 0; q < W; ++q)
      cl[r][q] = (ELL && q < a.W) ? a.cols[(size_t)q * a.d + row[r]] : row[r];
}

// ... and of control g0 + v - 1's entry qq, for the top blocks v >= 1.
template <int RPT, int V, int WK, bool ELL>
__device__ __forceinline__ void load_colk(const SweepArgs& a, int g0, const int (&row)[RPT],
                                          int (&ck)[V][RPT][WK]) {
#pragma unroll
  for (int v = 0; v < V; ++v)
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int q = 0; q < WK; ++q) {
        const int k = g0 + v - 1;
        ck[v][r][q] = (ELL && v >= 1 && k < a.K && q < a.WK[k])
                          ? a.colk[((size_t)k * kMaxDiagCtrl + q) * a.d + row[r]]
                          : row[r];
      }
}

// E_k/s = -i (dt/s) H_k on the control's own diagonals (FP64 -> working precision).
// ER (every control real or purely imaginary): the real factor e_k of
// E_k = w_k e_k instead (w_k = -i for a real H_k, 1 for an imaginary one), in .re.
template <typename R, int RPT, int WK, bool ER = false>
__device__ __forceinline__ void load_E(const SweepArgs& a, const double2* valk, int k, bool active,
                                       const int (&row)[RPT], const bool (&ok)[RPT], double cs,
                                       cx<R> (&ek)[RPT][WK]) {
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = opaque(row[r]);
#pragma unroll
    for (int q = 0; q < WK; ++q) {
      double er = 0.0, ei = 0.0;
      if (active && q < a.WK[k] && ok[r]) {
        const double2 v = valk[((size_t)k * kMaxDiagCtrl + q) * a.d + i];
        if (ER) {
          er = cs * (a.ecl[k] ? v.y : v.x);
        } else {
          er = cs * v.y;
          ei = -cs * v.x;
        }
      }
      ek[r][q] = cx<R>{(R)er, (R)ei};
    }
  }
}

// 1/j for the Taylor recursion, read through the scalar cache (uniform index).
__constant__ float kInvF[kMMax + 1] = {
    0.f,         1.f,         1.f / 2,  1.f / 3,  1.f / 4,  1.f / 5,  1.f / 6,  1.f / 7,
    1.f / 8,     1.f / 9,     1.f / 10, 1.f / 11, 1.f / 12, 1.f / 13, 1.f / 14, 1.f / 15,
    1.f / 16,    1.f / 17,    1.f / 18, 1.f / 19, 1.f / 20, 1.f / 21, 1.f / 22, 1.f / 23,
    1.f / 24,    1.f / 25,    1.f / 26, 1.f / 27, 1.f / 28, 1.f / 29, 1.f / 30, 1.f / 31,
    1.f / 32,    1.f / 33,    1.f / 34, 1.f / 35, 1.f / 36, 1.f / 37, 1.f / 38, 1.f / 39,
    1.f / 40,    1.f / 41,    1.f / 42, 1.f / 43, 1.f / 44, 1.f / 45, 1.f / 46, 1.f / 47,
    1.f / 48,    1.f / 49,    1.f / 50, 1.f / 51, 1.f / 52, 1.f / 53, 1.f / 54, 1.f / 55,
    1.f / 56,    1.f / 57,    1.f / 58, 1.f / 59, 1.f / 60};
__constant__ double kInvD[kMMax + 1] = {
    0.,        1.,        1. / 2,  1. / 3,  1. / 4,  1. / 5,  1. / 6,  1. / 7,  1. / 8,
    1. / 9,    1. / 10,   1. / 11, 1. / 12, 1. / 13, 1. / 14, 1. / 15, 1. / 16, 1. / 17,
    1. / 18,   1. / 19,   1. / 20, 1. / 21, 1. / 22, 1. / 23, 1. / 24, 1. / 25, 1. / 26,
    1. / 27,   1. / 28,   1. / 29, 1. / 30, 1. / 31, 1. / 32, 1. / 33, 1. / 34, 1. / 35,
    1. / 36,   1. / 37,   1. / 38, 1. / 39, 1. / 40, 1. / 41, 1. / 42, 1. / 43, 1. / 44,
    1. / 45,   1. / 46,   1. / 47, 1. / 48, 1. / 49, 1. / 50, 1. / 51, 1. / 52, 1. / 53,
    1. / 54,   1. / 55,   1. / 56, 1. / 57, 1. / 58, 1. / 59, 1. / 60};

template <typename R>
__device__ __forceinline__ R inv_const(int j);
template <>
__device__ __forceinline__ float inv_const<float>(int j) { return kInvF[j]; }
template <>
__device__ __forceinline__ double inv_const<double>(int j) { return kInvD[j]; }

// The kernels copy the table into LDS (after the reduction scratch) at start
// and read 1/j from there inside the term loop: a scalar-memory load in flight
// would share the LDS wait counter and force every pipelined gather of the term
// to wait for it (scalar loads return out of order).
constexpr int kInvOff = 512;
static_assert(kInvOff + (kMMax + 1) * 8 <= 1024, "1/j table must fit the LDS scratch");
template <typename R>
__device__ __forceinline__ void inv_table_to_lds(unsigned char* smem) {
  if ((int)threadIdx.x <= kMMax)
    reinterpret_cast<R*>(smem + kInvOff)[threadIdx.x] = inv_const<R>((int)threadIdx.x);
}

// ---------------------------------------------------------- LDS state block --
// A double-buffered block of V vectors is stored as planes of 16-byte rows:
// a plane row holds VP = 16/sizeof(complex) vectors of one matrix row (two
// complex64 or one complex128; a single complex64 vector uses 8-byte rows).
// Consecutive lanes own consecutive rows, so one ds_read of a plane row per
// (row, diagonal) is a contiguous, bank-conflict-free wave access.  Planes of
// a buffer are PS rows apart.  The layout parameter `rpt` here counts rows per
// 512 threads (a 1024-thread kernel with RPT rows per thread uses 2*RPT):
// PS = rpt * 512, the largest dimension for that count, when rpt <= 4 (a
// compile-time constant, so plane offsets fold into the instruction's
// immediate offset), else the dimension itself (runtime).  Reads at row + off
// outside [0, d) land in a neighbouring plane or in a zeroed guard of `halo`
// rows before the first and after the last plane: finite data times a zero
// coefficient (the operator diagonals are zero outside the matrix), so no
// bounds tests are needed.
__host__ __device__ constexpr int plane_rows(int rpt, int d) { return rpt <= 4 ? rpt * kMaxThreads : d; }
__host__ __device__ constexpr int block_vp(int cs, int v) { return (16 / cs) < v ? (16 / cs) : v; }
// Bytes of LDS of a double-buffered block of v vectors (both guards included).
__host__ __device__ constexpr int block_bytes(int cs, int rpt, int v, int d, int halo) {
  return 2 * ((v + block_vp(cs, v) - 1) / block_vp(cs, v)) * plane_rows(rpt, d) *
             (block_vp(cs, v) * cs) +
         2 * halo * block_vp(cs, v) * cs;
}

template <typename R, int RPT, int V>
struct Blk {
  static constexpr int CS = (int)sizeof(cx<R>);
  static constexpr int VP = block_vp(CS, V);
  static constexpr int NP = (V + VP - 1) / VP;
  static constexpr int RB = VP * CS;                 // bytes per plane row
  static constexpr bool CPS = RPT <= 4;              // compile-time plane stride?
  static constexpr int PSC = RPT * kMaxThreads * RB;  // that stride in bytes
  __device__ static uint32_t ps(int d) { return CPS ? (uint32_t)PSC : (uint32_t)d * RB; }
  __device__ static uint32_t bs(int d) { return NP * ps(d); }
  __device__ static int bytes(int d, int halo) { return block_bytes(CS, RPT, V, d, halo); }
  struct alignas(RB) Row {
    cx<R> v[VP];
  };
};

extern __shared__ __align__(16) unsigned char hg_smem[];

template <typename T>
__device__ __forceinline__ T lds_ld(uint32_t off) {
  return *reinterpret_cast<const T*>(hg_smem + off);
}
template <typename T>
__device__ __forceinline__ void lds_st(uint32_t off, const T& v) {
  *reinterpret_cast<T*>(hg_smem + off) = v;
}

// ------------------------------------------------------- split columns ------
// A column split over P workgroups (one per part, local columns h*P + part)
// refreshes the halo rows of every Taylor term from its neighbours.  Wave 0 of
// each workgroup copies its edge rows to global memory, publishes the exchange
// number with a release store at device scope, waits (bounded) until both
// neighbours have published it, and copies their edge rows into its halo rows;
// a barrier then hands the block to every wave.  Edge rows are double buffered
// by exchange parity: a neighbour can be at most one exchange ahead.  A wait
// that exceeds a.xwait (or sees another workgroup's timeout) sets the error
// flag and stops all further waiting of this workgroup, which then finishes
// its sweep with meaningless numbers; the host reports the error.
struct XState {
  int b, hp, part;   // evaluation, local column, part
  uint32_t seq;      // exchanges so far (the same in every part of a column)
  int abort;         // (wave 0) a wait failed: no more waiting
};

__device__ __forceinline__ bool xwait(const SweepArgs& a, int col, uint32_t seq, uint64_t t0) {
  while (__hip_atomic_load(&a.xflag[col], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < seq) {
    if (__hip_atomic_load(a.xerr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    if (__builtin_amdgcn_s_memrealtime() - t0 > a.xwait) {
      __hip_atomic_store(a.xerr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

template <typename R, int LR, int V>
__device__ __forceinline__ void halo_exchange(const SweepArgs& a, uint32_t base, uint32_t buf,
                                           XState& xs) {
  using L = Blk<R, LR, V>;
  using Row = typename L::Row;
  static_assert(L::NP * L::RB <= kXRowBytes, "exchange row too wide");
  if (a.xh == 0) return;  // parts share no rows: nothing to exchange
  xs.seq += 1u;
  if (threadIdx.x < 64 && !xs.abort) {
    const int lane = threadIdx.x;
    const int hh = a.xh, seg = a.xseg, w = a.xw[xs.part], ne = a.xrows, d = a.d;
    const uint32_t slot = xs.seq & 1u;
    const int col = xs.b * a.S + xs.hp;
    auto xrow = [&](int c, uint32_t sl, int side, int r) {
      return a.xbuf + ((((size_t)c * 2 + sl) * 2 + side) * ne + r) * kXRowBytes;
    };
    // side 0: the first hh own rows of every block, side 1: the last hh
    for (int i = lane; i < 2 * ne * L::NP; i += 64) {
      const int pl = i % L::NP, r = (i / L::NP) % ne, side = i / (L::NP * ne);
      const int t = r / hh, k = r % hh;
      const uint32_t lrow = (uint32_t)(t * seg + (side == 0 ? hh + k : w + k));
      const Row v = lds_ld<Row>(base + buf + lrow * L::RB + pl * L::ps(d));
      *reinterpret_cast<Row*>(xrow(col, slot, side, r) + pl * L::RB) = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(&a.xflag[col], xs.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    if (lane == 0) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      if (xs.part > 0 && !xwait(a, col - 1, xs.seq, t0)) ok = 0;
      if (ok && xs.part + 1 < a.P && !xwait(a, col + 1, xs.seq, t0)) ok = 0;
    }
    ok = __builtin_amdgcn_readfirstlane(ok);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (!ok) {
      xs.abort = 1;
    } else {
      // left neighbour's side 1 -> my low halo rows; right neighbour's side 0 -> my high halo rows
      for (int i = lane; i < 2 * ne * L::NP; i += 64) {
        const int pl = i % L::NP, r = (i / L::NP) % ne, side = i / (L::NP * ne);
        const int t = r / hh, k = r % hh;
        if (side == 0 ? xs.part == 0 : xs.part + 1 == a.P) continue;
        const unsigned char* src = side == 0 ? xrow(col - 1, slot, 1, r) : xrow(col + 1, slot, 0, r);
        const uint32_t lrow = (uint32_t)(t * seg + (side == 0 ? k : hh + w + k));
        lds_st(base + buf + lrow * L::RB + pl * L::ps(d), *reinterpret_cast<const Row*>(src + pl * L::RB));
      }
    }
  }
  __syncthreads();
}

// Sum of one value over the P parts of this column, in part order (so every
// part gets the same bits).  All threads call it; the result goes to all.
__device__ __forceinline__ double part_allsum(const SweepArgs& a, double v, XState& xs, double* red) {
  xs.seq += 1u;
  if (threadIdx.x < 64 && !xs.abort) {
    const int lane = threadIdx.x;
    const int col = xs.b * a.S + xs.hp, first = col - xs.part;
    const uint32_t slot = xs.seq % (uint32_t)kMaxParts;
    if (lane == 0) {
      a.xnrm[(size_t)col * kMaxParts + slot] = v;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&a.xflag[col], xs.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    if (lane == 0) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      for (int q = 0; q < a.P && ok; ++q)
        if (q != xs.part && !xwait(a, first + q, xs.seq, t0)) ok = 0;
    }
    ok = __builtin_amdgcn_readfirstlane(ok);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (!ok) {
      xs.abort = 1;
    } else if (lane == 0) {
      double t = 0.0;
      for (int q = 0; q < a.P; ++q) t += a.xnrm[(size_t)(first + q) * kMaxParts + slot];
      red[60] = t;
    }
  }
  __syncthreads();
  const double t = red[60];
  __syncthreads();
  return xs.abort && threadIdx.x < 64 ? v : t;
}

// Tail-vector role of a wavefront (see taylor_block): kNotShared for a wave
// that keeps its own last row slab, else the vector it computes on the shared
// slab (-1: none).
constexpr int kNotShared = -2;

// Write the V accumulators of this thread's rows into buffer 0 of the block.
// On a wave of the shared tail slab the last row carries only vector tv
// (none if tv < 0), written on its own.
template <typename R, int RPT, int V, int LR = RPT, typename A = R>
__device__ __forceinline__ void block_store(uint32_t base, int d, const uint32_t (&rowb)[RPT],
                                            const bool (&ok)[RPT], int tv,
                                            const cx<A> (&acc)[RPT][V]) {
  using L = Blk<R, LR, V>;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (tv != kNotShared && r == RPT - 1) {
      if (tv >= 0 && ok[r]) {
        // select, then round: converting inside the selection makes the
        // compiler index acc dynamically and move it to scratch memory
        cx<A> y = acc[r][0];
#pragma unroll
        for (int v = 1; v < V; ++v)
          if (tv == v) y = acc[r][v];
        const cx<R> x = cxc<R>(y);
        lds_st(base + rowb[r] + (uint32_t)(tv / L::VP) * L::ps(d) + (uint32_t)(tv % L::VP) * L::CS, x);
      }
      continue;
    }
    if (ok[r])
#pragma unroll
      for (int p = 0; p < L::NP; ++p) {
        typename L::Row w;
#pragma unroll
        for (int q = 0; q < L::VP; ++q)
          w.v[q] = (p * L::VP + q < V) ? cxc<R>(acc[r][p * L::VP + q]) : cx<R>{(R)0, (R)0};
        lds_st(base + rowb[r] + p * L::ps(d), w);
      }
  }
}

// One Taylor term for the V vectors of this thread's rows, reading buffer
// SRC1 and writing the other one:
//   t^v = sgn/j * (sum_e B[r][e] src^v[row + off_e]  (+ E_k/s src^Y[row + offk] for AUX tops))
//   acc += t ; dst = t
// The gathers are software-pipelined: a ring of PD+1 register slots keeps PD
// LDS reads in flight ahead of the FMAs that consume them, and a scheduling
// barrier after each item pins that order.  Items run row by row: first the W
// union diagonals (NP plane-row reads each), then for AUX the (V-1)*WK
// derivative operand reads (the Y entry only).  Each gather address is one
// add of a per-row base (VGPR) and the diagonal's offset (SGPR); keeping all
// RPT*W addresses in registers instead spills at these register budgets and
// did not make the forward kernel faster.
template <typename R, int RPT, int NR, int W, int PU, int V, int WK, bool AUX, bool SRC1, int LR = RPT,
          typename A = R>
__device__ __forceinline__ void taylor_term(uint32_t base, const SweepArgs& a, int g0,
                                            const uint32_t (&rowb)[RPT], const bool (&ok)[RPT],
                                            const cx<R> (&bv)[RPT][W],
                                            const cx<R> (&ek)[V][RPT][WK],
                                            const int (&cl)[RPT][W], const int (&ckl)[V][RPT][WK], R inv,
                                            cx<A> (&acc)[RPT][V]) {
  using C = cx<R>;
  using L = Blk<R, LR, V>;
  using Row = typename L::Row;
  constexpr bool ELL = (PU & 8) != 0;  // row-indexed storage: per-row gather columns
  constexpr int NIR = W + (AUX ? (V - 1) * WK : 0);
  constexpr int NI = NR * NIR;  // only the first NR rows (a wave's last slab may be empty)
  constexpr int PD = V == 1 ? (sizeof(R) == 4 ? 6 : 3) : (V == 2 && sizeof(R) == 4 ? 3 : 2);
  constexpr int NS = PD + 1;
  const int d = a.d;
  const uint32_t SRC = SRC1 ? L::bs(d) : 0, DST = SRC1 ? 0 : L::bs(d);
  Row ring[NS][L::NP];
  C t[V];
  uint32_t rb[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) rb[r] = V > 1 ? (uint32_t)opaque((int)rowb[r]) : rowb[r];
#pragma unroll
  for (int it = 0; it < NI + PD; ++it) {
    if (it < NI) {  // issue the gather of item `it`
      const int r = it / NIR, q = it % NIR;
      if (q < W) {
        const uint32_t ad =
            ELL ? (uint32_t)opaque(cl[r][q]) * (uint32_t)L::RB + opaque_s(base + SRC)
                : rb[r] + opaque_s((uint32_t)(a.off[q] * L::RB) + base + SRC);
#pragma unroll
        for (int p = 0; p < L::NP; ++p) ring[it % NS][p] = lds_ld<Row>(ad + p * L::ps(d));
      } else {
        const int v = 1 + (q - W) / WK, qq = (q - W) % WK;
        const int kk = g0 + v - 1 < a.K ? g0 + v - 1 : 0;
        ring[it % NS][0].v[0] = lds_ld<C>(
            ELL ? (uint32_t)opaque(ckl[v][r][qq]) * (uint32_t)L::RB + opaque_s(base + SRC)
                : rb[r] + opaque_s((uint32_t)(a.offk[kk][qq] * L::RB) + base + SRC));
      }
    }
    if (it >= PD) {  // consume item `it - PD`
      const int c = it - PD;
      const int r = c / NIR, q = c % NIR;
      if (q == 0) {
#pragma unroll
        for (int v = 0; v < V; ++v) t[v] = C{(R)0, (R)0};
      }
      if (q < W) {
#pragma unroll
        for (int v = 0; v < V; ++v) bmac<PU>(q, t[v], bv[r][q], ring[c % NS][v / L::VP].v[v % L::VP]);
      } else {
        const int v = 1 + (q - W) / WK, qq = (q - W) % WK;
        emac<PU>(t[v], ek[v][r][qq], ring[c % NS][0].v[0]);
      }
      if (q == NIR - 1) {  // row complete
#pragma unroll
        for (int v = 0; v < V; ++v) {
          t[v].re *= inv;
          t[v].im *= inv;
          acc[r][v].re += t[v].re;
          acc[r][v].im += t[v].im;
        }
        if (ok[r])
#pragma unroll
          for (int p = 0; p < L::NP; ++p) {
            Row w;
#pragma unroll
            for (int qv = 0; qv < L::VP; ++qv)
              w.v[qv] = (p * L::VP + qv < V) ? t[p * L::VP + qv] : C{(R)0, (R)0};
            lds_st(rb[r] + opaque_s(base + DST) + p * L::ps(d), w);
          }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The shared tail slab's share of one Taylor term: vector VT of the last row
// (RPT-1) only, with the same products as taylor_term for that vector.
template <typename R, int RPT, int W, int PU, int V, int WK, bool AUX, bool SRC1, int VT, int LR,
          typename A>
__device__ __forceinline__ void tail_piece(uint32_t base, const SweepArgs& a, int g0,
                                           const uint32_t (&rowb)[RPT], const bool (&ok)[RPT],
                                           const cx<R> (&bv)[RPT][W],
                                           const cx<R> (&ek)[V][RPT][WK],
                                           const int (&cl)[RPT][W], const int (&ckl)[V][RPT][WK], R inv,
                                           cx<A> (&acc)[RPT][V]) {
  using C = cx<R>;
  using L = Blk<R, LR, V>;
  constexpr int r = RPT - 1;
  const int d = a.d;
  const uint32_t SRC = SRC1 ? L::bs(d) : 0, DST = SRC1 ? 0 : L::bs(d);
  const uint32_t vo = (uint32_t)(VT / L::VP) * L::ps(d) + (uint32_t)(VT % L::VP) * L::CS;
  const uint32_t rb = (uint32_t)opaque((int)rowb[r]);
  C x[W];
  constexpr bool ELL = (PU & 8) != 0;
#pragma unroll
  for (int q = 0; q < W; ++q)
    x[q] = lds_ld<C>((ELL ? (uint32_t)opaque(cl[r][q]) * (uint32_t)L::RB + opaque_s(base + SRC)
                          : rb + opaque_s((uint32_t)(a.off[q] * L::RB) + base + SRC)) + vo);
  C y[(AUX && VT > 0) ? WK : 1];
  if constexpr (AUX && VT > 0) {
    const int kk = g0 + VT - 1 < a.K ? g0 + VT - 1 : 0;
#pragma unroll
    for (int q = 0; q < WK; ++q)
      y[q] = lds_ld<C>(ELL ? (uint32_t)opaque(ckl[VT][r][q]) * (uint32_t)L::RB + opaque_s(base + SRC)
                           : rb + opaque_s((uint32_t)(a.offk[kk][q] * L::RB) + base + SRC));
  }
  C t{(R)0, (R)0};
#pragma unroll
  for (int q = 0; q < W; ++q) bmac<PU>(q, t, bv[r][q], x[q]);
  if constexpr (AUX && VT > 0) {
#pragma unroll
    for (int q = 0; q < WK; ++q) emac<PU>(t, ek[VT][r][q], y[q]);
  }
  t.re *= inv;
  t.im *= inv;
  acc[r][VT].re += t.re;
  acc[r][VT].im += t.im;
  if (ok[r]) lds_st(rb + opaque_s(base + DST) + vo, t);
}

template <typename R, int RPT, int W, int PU, int V, int WK, bool AUX, bool SRC1, int LR, typename A>
__device__ __forceinline__ void tail_share(int tv, uint32_t base, const SweepArgs& a, int g0,
                                           const uint32_t (&rowb)[RPT], const bool (&ok)[RPT],
                                           const cx<R> (&bv)[RPT][W],
                                           const cx<R> (&ek)[V][RPT][WK],
                                           const int (&cl)[RPT][W], const int (&ckl)[V][RPT][WK], R inv,
                                           cx<A> (&acc)[RPT][V]) {
  switch (tv) {
    case 0:
      tail_piece<R, RPT, W, PU, V, WK, AUX, SRC1, 0, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, inv, acc);
      break;
    case 1:
      if constexpr (V > 1) tail_piece<R, RPT, W, PU, V, WK, AUX, SRC1, 1, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, inv, acc);
      break;
    case 2:
      if constexpr (V > 2) tail_piece<R, RPT, W, PU, V, WK, AUX, SRC1, 2, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, inv, acc);
      break;
    case 3:
      if constexpr (V > 3) tail_piece<R, RPT, W, PU, V, WK, AUX, SRC1, 3, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, inv, acc);
      break;
    default:
      break;
  }
}

// One application of (T_m(sgn*B))^s to the V vectors held in `acc`:
//   t_0 = acc, t_j = (sgn B / j) t_{j-1}, acc += t_j   (Sec. III.B, eq. eBmpsi)
// repeated s times (scaling and squaring, eq. scaling squaring).  With AUX,
// vectors 1..V-1 are the top blocks X_k of the auxiliary vector (X_k; Y) with
// Y = vector 0, i.e. t_j^X += (E_k/s / j) t_{j-1}^Y (eq. auxiliary equation).
// `base` is the byte offset of buffer 0, plane 0, row 0.  The term loop is
// unrolled by two so the buffer being read is a compile-time choice.  Ends
// with a barrier, so the block may be rewritten right away.
template <typename R, int RPT, int W, int PU, int V, int WK, bool AUX, int LR, bool SPLIT, typename A>
__device__ __forceinline__ void taylor_block(uint32_t base, const SweepArgs& a, int g0,
                                             const uint32_t (&rowb)[RPT],
                                             const bool (&ok)[RPT], const bool (&sv)[RPT],
                                             int tv,
                                             const cx<R> (&bv)[RPT][W],
                                             const cx<R> (&ek)[V][RPT][WK],
                                             const int (&cl)[RPT][W], const int (&ckl)[V][RPT][WK],
                                             int m, int s, R sgn,
                                             cx<A> (&acc)[RPT][V], XState& xs) {
  // A wavefront whose last row slab lies past the dimension runs the RPT-1 row
  // variant (wave-uniform choice, both variants fully unrolled).  The waves of
  // a shared tail slab (tv != kNotShared: four waves on different SIMDs) run
  // RPT-1 rows and split that slab by vector: vector tv by this one (V == 1:
  // the whole slab if tv == 0).
  const bool full = tv == kNotShared ? sv[RPT - 1] : (V == 1 && tv == 0);
  const bool share = sizeof(R) == 4 && V > 1 && tv >= 0;
  constexpr int NRS = RPT > 1 ? RPT - 1 : 1;
  using BL = Blk<R, LR, V>;
  for (int l = 0; l < s; ++l) {
    block_store<R, RPT, V, LR, A>(base, a.d, rowb, ok, tv, acc);
    __syncthreads();
    if constexpr (SPLIT) halo_exchange<R, LR, V>(a, base, 0u, xs);
    for (int j = 1; j <= m; j += 2) {
      const R i1 = sgn * lds_ld<R>(kInvOff + j * (int)sizeof(R));
      if (full)
        taylor_term<R, RPT, RPT, W, PU, V, WK, AUX, false, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, i1, acc);
      else
        taylor_term<R, RPT, NRS, W, PU, V, WK, AUX, false, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, i1, acc);
      if (share) tail_share<R, RPT, W, PU, V, WK, AUX, false, LR, A>(tv, base, a, g0, rowb, ok, bv, ek, cl, ckl, i1, acc);
      __syncthreads();
      if constexpr (SPLIT) halo_exchange<R, LR, V>(a, base, BL::bs(a.d), xs);
      if (j + 1 <= m) {
        const R i2 = sgn * lds_ld<R>(kInvOff + (j + 1) * (int)sizeof(R));
        if (full)
          taylor_term<R, RPT, RPT, W, PU, V, WK, AUX, true, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, i2, acc);
        else
          taylor_term<R, RPT, NRS, W, PU, V, WK, AUX, true, LR, A>(base, a, g0, rowb, ok, bv, ek, cl, ckl, i2, acc);
        if (share) tail_share<R, RPT, W, PU, V, WK, AUX, true, LR, A>(tv, base, a, g0, rowb, ok, bv, ek, cl, ckl, i2, acc);
        __syncthreads();
        if constexpr (SPLIT) halo_exchange<R, LR, V>(a, base, 0u, xs);
      }
    }
  }
}

template <int RPT, bool SPLIT>
__device__ __forceinline__ void renormalise(CA (&p)[RPT], double* red, const SweepArgs& a,
                                            XState& xs) {
  double nv[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r) nv[0] = acc_norm2(nv[0], p[r]);
  block_sum<1>(nv, red);
  if constexpr (SPLIT) nv[0] = part_allsum(a, nv[0], xs, red);
  const double sc = 1.0 / sqrt(nv[0]);
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    p[r].re *= sc;
    p[r].im *= sc;
  }
}

// ---------------------------------------------------------------- forward ----
// psi_n = (T_m(B_n))^s psi_{n-1} for n = 1..N (Sec. III.B, eq. eBmpsi);
// penalty partial sum_n <psi_n|Omega|psi_n> (App. A, eq. c2st) and the overlap
// <phi_T|psi_N> (Sec. III.A) of this column.
// TPB threads per workgroup; the LDS layout is that of LR = RPT*TPB/512 rows
// per 512 threads, so the forward can run 1024 threads (4 waves per SIMD, to
// hide the latency of its short, barrier-separated terms).
template <typename R, int RPT, int W, int PU, int TPB, bool SPLIT, int CPW = 1>
__global__ void __launch_bounds__(TPB) hg_forward(SweepArgs a) {
  // CPW state columns of one evaluation per workgroup (CPW = 2: the columns
  // share B_n, the gather addresses and each term's barrier, and read their
  // operands pairwise; used when the launch still fills the chip)
  static_assert(CPW == 1 || !SPLIT, "split columns run one column per workgroup");
  using C = cx<R>;
  constexpr int LR = RPT * TPB / kMaxThreads;
  using L = Blk<R, LR, CPW>;
  double* red = reinterpret_cast<double*>(hg_smem);
  const int d = a.d, tid = threadIdx.x, NT = blockDim.x;
  const int h = blockIdx.x * CPW, b = blockIdx.y;
  size_t col0[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) col0[c] = ((size_t)b * a.S + h + c) * d;
  // a split column's part: its slice of the local operators
  const int part = SPLIT ? h % a.P : 0;
  const double2* vals = a.vals + (SPLIT ? (size_t)part * a.psv : 0);
  const double* omega = a.omega ? a.omega + (SPLIT ? (size_t)part * a.pso : 0) : nullptr;
  XState xs{b, h, part, 0u, 0};
  {
    uint32_t* z = reinterpret_cast<uint32_t*>(hg_smem + kRedBytes);
    for (int i = tid; i < L::bytes(d, a.halo) / 4; i += NT) z[i] = 0u;
    inv_table_to_lds<R>(hg_smem);
  }
  const uint32_t base = kRedBytes + a.halo * L::RB;

  int row[RPT];
  uint32_t rowb[RPT];
  bool ok[RPT], sv[RPT];
  slab_valid<RPT>(d, sv);
  CA acc[RPT][CPW];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * NT;
    ok[r] = i < d;
    row[r] = ok[r] ? i : d - 1;
    rowb[r] = (uint32_t)row[r] * L::RB;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double2 p = a.psi0[col0[c] + row[r]];
      acc[r][c] = ok[r] ? CA{p.x, p.y} : CA{0.0, 0.0};
    }
  }
  __syncthreads();

  C ek[CPW][RPT][1];
  int cl[RPT][W], ckf[CPW][RPT][1];
  load_cols<RPT, W, (PU & 8) != 0>(a, row, cl);
  load_colk<RPT, CPW, 1, false>(a, 0, row, ckf);
  double pen[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) pen[c] = 0.0;
  const double* ub = a.u + (size_t)b * a.K * a.N;
  const int CK = a.ckpt_every;
  C* ck[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    ck[c] = CK > 0 ? reinterpret_cast<C*>(a.ckpt) +
                         ((size_t)b * a.S + h + c) * (size_t)((a.N + CK - 1) / CK) * d
                   : nullptr;
    if (ck[c])
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (ok[r]) ck[c][row[r]] = cxc<R>(acc[r][c]);
  }
  for (int n = 0; n < a.N; ++n) {
    const int m = a.msch[(size_t)b * a.N + n];
    const int s = a.ssch[(size_t)b * a.N + n];
    C bv[RPT][W];
    assemble_B<R, RPT, W>(a, vals, ub, n, row, ok, a.dt / (double)s, bv);
    taylor_block<R, RPT, W, PU, CPW, 1, false, LR, SPLIT>(base, a, 0, rowb, ok, sv, kNotShared, bv,
                                                      ek, cl, ckf, m, s, (R)1, acc, xs);
    if (a.renorm_every > 0 && (n + 1) % a.renorm_every == 0) {
      if constexpr (SPLIT) {
        CA p[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) p[r] = acc[r][0];
        renormalise<RPT, SPLIT>(p, red, a, xs);
#pragma unroll
        for (int r = 0; r < RPT; ++r) acc[r][0] = p[r];
      } else {
        double nv[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          nv[c] = 0.0;
#pragma unroll
          for (int r = 0; r < RPT; ++r) nv[c] = acc_norm2(nv[c], acc[r][c]);
        }
        block_sum<CPW>(nv, red);
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          const double sc = 1.0 / sqrt(nv[c]);
#pragma unroll
          for (int r = 0; r < RPT; ++r) {
            acc[r][c].re *= sc;
            acc[r][c].im *= sc;
          }
        }
      }
    }
    if (omega) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (ok[r])
#pragma unroll
          for (int c = 0; c < CPW; ++c)
            pen[c] = fma(omega[row[r]], acc_norm2(0.0, acc[r][c]), pen[c]);
    }
    if (CK > 0 && (n + 1) % CK == 0 && n + 1 < a.N)
#pragma unroll
      for (int c = 0; c < CPW; ++c)
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (ok[r]) ck[c][(size_t)((n + 1) / CK) * d + row[r]] = cxc<R>(acc[r][c]);
    if (a.ovt) {
      // <phi_T|psi_{n+1}> of each column for the time-integrated infidelity
      double o[2 * CPW];
#pragma unroll
      for (int q = 0; q < 2 * CPW; ++q) o[q] = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (ok[r])
#pragma unroll
          for (int c = 0; c < CPW; ++c) {
            acc_dot(o[2 * c + 0], o[2 * c + 1], a.tgt[col0[c] + row[r]], acc[r][c]);
          }
      block_sum<2 * CPW>(o, red);
      if (tid == 0)
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          a.ovt[(((size_t)b * a.S + h + c) * a.N + n) * 2 + 0] = o[2 * c + 0];
          a.ovt[(((size_t)b * a.S + h + c) * a.N + n) * 2 + 1] = o[2 * c + 1];
        }
    }
  }

  C* psiN = reinterpret_cast<C*>(a.psiN);
  // one column at a time: the reduction scratch holds at most 4 sums
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    double v[3] = {0.0, 0.0, pen[c]};
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (ok[r]) {
        psiN[col0[c] + row[r]] = cxc<R>(acc[r][c]);
        acc_dot(v[0], v[1], a.tgt[col0[c] + row[r]], acc[r][c]);  // conj(phi) psi
      }
    block_sum<3>(v, red);
    if (tid == 0) {
      a.ovl[((size_t)b * a.S + h + c) * 2 + 0] = v[0];
      a.ovl[((size_t)b * a.S + h + c) * 2 + 1] = v[1];
      a.pen[(size_t)b * a.S + h + c] = v[2];
    }
  }
}

// --------------------------------------------------------------- backward ----
// For n = N..1 (kernel index n-1):
//   psi_{n-1}   = (T_m(-B_n))^s psi_n           inverse propagation (Sec. III.C)
//   Lambda'     = (T_m(-B_n))^s Lambda_n        co-state, U^dag = T(B^dag) = T(-B)
//   (X_k; Y)    = (T_m(Aux_k/s))^s (0; psi_{n-1}), Aux_k = [[A, E_k],[0, A]]
//                                                (Sec. III.B, eq. auxiliary equation)
//   grad[k][n]  = 2 Re <Lambda_n | X_k>          (Sec. III.A, App. A)
//   Lambda_{n-1} = Lambda' + (w_pen/(N S)) Omega psi_{n-1}   for n-1 >= 1 (App. A)
// Controls are processed in groups of G (the bottom block Y is recomputed per
// group) so that the (1+G)-vector double-buffered block fits in LDS.
// TPB threads per workgroup, LDS layout of LR = RPT*TPB/512 rows per 512
// threads (as in the forward kernel).
template <typename R, int RPT, int W, int PU, int WK, int G, int TPB, bool SPLIT>
__global__ void __launch_bounds__(TPB) hg_backward(SweepArgs a) {
  using C = cx<R>;
  constexpr int V2 = 1 + G;
  constexpr int LR = RPT * TPB / kMaxThreads;
  using L1 = Blk<R, LR, 2>;
  using L2 = Blk<R, LR, V2>;
  double* red = reinterpret_cast<double*>(hg_smem);
  const int d = a.d, tid = threadIdx.x, NT = blockDim.x, K = a.K, N = a.N, S = a.S;
  const int h = blockIdx.x, b = blockIdx.y;
  const size_t col0 = ((size_t)b * S + h) * d;
  // a split column's part: its slice of the local operators; the cost is
  // normalised by the true number of states St (S counts local columns)
  const int part = SPLIT ? h % a.P : 0;
  const double2* vals = a.vals + (SPLIT ? (size_t)part * a.psv : 0);
  const double2* valk = a.valk + (SPLIT ? (size_t)part * a.psk : 0);
  const double* omega = a.omega ? a.omega + (SPLIT ? (size_t)part * a.pso : 0) : nullptr;
  const int St = a.St;
  XState xs{b, h, part, 0u, 0};
  {
    const int nb1 = L1::bytes(d, a.halo), nb2 = L2::bytes(d, a.halo);
    const int nb = nb1 > nb2 ? nb1 : nb2;
    uint32_t* z = reinterpret_cast<uint32_t*>(hg_smem + kRedBytes);
    for (int i = tid; i < nb / 4; i += NT) z[i] = 0u;
    inv_table_to_lds<R>(hg_smem);
  }
  // phase 1 block (psi, Lambda) and phase 2 block (Y, X_1..X_G) share the region
  const uint32_t base1 = kRedBytes + a.halo * L1::RB;
  const uint32_t base2 = kRedBytes + a.halo * L2::RB;

  // Several workgroups may share a column (gridDim.z = Q): each repeats the
  // reconstruction and co-state (phase 1) and takes every Q-th group of G
  // controls in phase 2, so a column's backward sweep spreads over Q compute
  // units.  The arithmetic of each control is the same whichever workgroup
  // runs it.  Rarely touched per-row vectors and checkpoint segments are per
  // workgroup; only z = 0 writes the cost parts and the drift.
  const int z = blockIdx.z, Q = gridDim.z;
  CA* cold = reinterpret_cast<CA*>(a.cold) + (((size_t)b * S + h) * Q + z) * 3 * d;
  CA* const c_psi = cold;          // psi_{n-1}
  CA* const c_lam = cold + d;      // propagated co-state
  // Lambda_n for the overlaps, in the working precision: it is used for one
  // step only, and the narrower copy keeps the per-step rows within the L2
  C* const c_cur = reinterpret_cast<C*>(cold + 2 * d);

  // Shared tail slab: the last plane of rows holds T slabs of 64 rows.  With
  // T = 4q+1 the last one (index ts = T-1) would leave one SIMD a slab more
  // than the others; instead waves ts..ts+3 (one per SIMD; their own slabs of
  // that plane lie past the dimension) all map their last row to it and own
  // one vector each there: psi -> ts, Lambda -> ts+1 in phase 1, Y -> ts and
  // X_v -> ts+v in phase 2.  A thread's copy of a tail vector it does not own
  // stays zero, so sums over rows need no extra test; stores are guarded.
  // (complex64 only: the complex128 kernels have no registers to spare for it)
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tail0 = (RPT - 1) * NT;
  const int T = d > tail0 ? (d - tail0 + 63) / 64 : 0;
  const int ts = T - 1;
  const bool split = sizeof(R) == 4 && RPT > 1 && T % 4 == 1 && ts + 4 <= NT / 64;
  const bool tailw = split && wv >= ts && wv < ts + 4;
  const int tw = wv - ts;  // this wave's index in the sharing group

  int row[RPT];
  uint32_t rowb1[RPT], rowb2[RPT];
  bool ok[RPT], sv[RPT], own_psi[RPT], own_lam[RPT];
  slab_valid<RPT>(d, sv);
  CA pl[RPT][2];  // psi and Lambda
  const C* psiN = reinterpret_cast<const C*>(a.psiN);

  // the turn: g, cost parts, Lambda_N = -(w_fid g/S) phi_T + (w_pen/(N S)) Omega psi_N
  double gre = 0.0, gim = 0.0, ptot = 0.0;
  for (int k = 0; k < S; ++k) {
    gre += a.ovl[((size_t)b * S + k) * 2 + 0];
    gim += a.ovl[((size_t)b * S + k) * 2 + 1];
    ptot += a.pen[(size_t)b * S + k];
  }
  gre /= (double)St;
  gim /= (double)St;
  const double cpen = omega ? a.w_pen / ((double)N * St) : 0.0;
  // time-integrated infidelity: C3 (written by k_integrated) and the source
  // -(w_int/(N S)) g_n phi_T of every state psi_n, n = N..1 (App. A, Phi_T,n)
  const double cint = a.ovt ? a.w_int / ((double)N * St) : 0.0;
  if (h == 0 && z == 0 && tid == 0) {
    const double C1 = 1.0 - (gre * gre + gim * gim);
    const double C2 = omega ? ptot / ((double)N * St) : 0.0;
    const double C3 = a.ovt ? a.res[(size_t)b * 8 + 5] : 0.0;
    a.res[(size_t)b * 8 + 0] =
        a.w_fid * C1 + (omega ? a.w_pen * C2 : 0.0) + (a.ovt ? a.w_int * C3 : 0.0);
    a.res[(size_t)b * 8 + 1] = C1;
    a.res[(size_t)b * 8 + 2] = C2;
    a.res[(size_t)b * 8 + 3] = gre;
    a.res[(size_t)b * 8 + 4] = gim;
    a.res[(size_t)b * 8 + 5] = C3;
  }
  const double fr = -(a.w_fid / St + cint) * gre, fi = -(a.w_fid / St + cint) * gim;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const bool shared = tailw && r == RPT - 1;
    const int i = shared ? tail0 + ts * 64 + (tid & 63) : tid + r * NT;
    ok[r] = i < d;
    own_psi[r] = ok[r] && (!shared || tw == 0);
    own_lam[r] = ok[r] && (!shared || tw == 1);
    row[r] = ok[r] ? i : d - 1;
    rowb1[r] = (uint32_t)row[r] * L1::RB;
    rowb2[r] = (uint32_t)row[r] * L2::RB;
    const C p = psiN[col0 + row[r]];
    const double2 t = a.tgt[col0 + row[r]];
    const double w = omega ? omega[row[r]] : 0.0;
    pl[r][0] = own_psi[r] ? cxc<double>(p) : CA{0.0, 0.0};
    pl[r][1].re = own_lam[r] ? fr * t.x - fi * t.y + cpen * w * (double)p.re : 0.0;
    pl[r][1].im = own_lam[r] ? fr * t.y + fi * t.x + cpen * w * (double)p.im : 0.0;
  }
  __syncthreads();
  // tail vector of this wavefront in the phase-1 block, the phase-2 block and
  // the single-vector blocks of psi and of Lambda
  const int tv1 = !tailw ? kNotShared : tw < 2 ? tw : -1;
  const int tv2 = !tailw ? kNotShared : tw < V2 ? tw : -1;
  const int tvp = !tailw ? kNotShared : tw == 0 ? 0 : -1;
  const int tvl = !tailw ? kNotShared : tw == 1 ? 0 : -1;

  C ek1[2][RPT][1];
  int cl[RPT][W], ck1[2][RPT][1], ckf[1][RPT][1];
  load_cols<RPT, W, (PU & 8) != 0>(a, row, cl);
  load_colk<RPT, 2, 1, false>(a, 0, row, ck1);
  load_colk<RPT, 1, 1, false>(a, 0, row, ckf);
  const double* ub = a.u + (size_t)b * K * N;
  // Reconstruction variant: one segment, psi_{n-1} rebuilt by (T_m(-B_n))^s.
  // Checkpoint variant: segments of CK steps swept back last to first; each is
  // first re-propagated forward from its stored psi (the same products as the
  // forward sweep), keeping its states, so only Lambda is propagated backwards.
  const bool ckpt = a.ckpt_every > 0;
  const int CK = ckpt ? a.ckpt_every : N;
  const int nseg = (N + CK - 1) / CK;
  using LF = Blk<R, LR, 1>;
  const uint32_t basef = kRedBytes + a.halo * LF::RB;
  uint32_t rowbf[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) rowbf[r] = (uint32_t)row[r] * LF::RB;
  const C* ckb = ckpt ? reinterpret_cast<const C*>(a.ckpt) + ((size_t)b * S + h) * (size_t)nseg * d
                      : nullptr;
  C* seg = ckpt ? reinterpret_cast<C*>(a.segbuf) + (((size_t)b * S + h) * Q + z) * (size_t)CK * d
                 : nullptr;
  for (int sg = nseg - 1; sg >= 0; --sg) {
  const int n0 = ckpt ? sg * CK : 0;
  const int n1 = ckpt ? (n0 + CK < N ? n0 + CK : N) : N;
  if (ckpt) {
    CA f[RPT][1];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      f[r][0] = own_psi[r] ? cxc<double>(ckb[(size_t)sg * d + row[r]]) : CA{0.0, 0.0};
    for (int n = n0; n < n1; ++n) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (own_psi[r]) seg[(size_t)(n - n0) * d + opaque(row[r])] = cxc<R>(f[r][0]);
      const int m = a.msch[(size_t)b * N + n];
      const int s = a.ssch[(size_t)b * N + n];
      C bv[RPT][W];
      assemble_B<R, RPT, W>(a, vals, ub, n, row, ok, a.dt / (double)s, bv);
      C ekf[1][RPT][1];
      taylor_block<R, RPT, W, PU, 1, 1, false, LR, SPLIT>(basef, a, 0, rowbf, ok, sv, tvp, bv, ekf,
                                                      cl, ckf, m, s, (R)1, f, xs);
      if (a.renorm_every > 0 && (n + 1) % a.renorm_every == 0) {
        CA p[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) p[r] = f[r][0];
        renormalise<RPT, SPLIT>(p, red, a, xs);
#pragma unroll
        for (int r = 0; r < RPT; ++r) f[r][0] = p[r];
      }
    }
  }
  for (int n = n1 - 1; n >= n0; --n) {
    const int m = a.msch[(size_t)b * N + n];
    const int s = a.ssch[(size_t)b * N + n];
    const double cs = a.dt / (double)s;
    C bv[RPT][W];
    assemble_B<R, RPT, W>(a, vals, ub, n, row, ok, cs, bv);
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (own_lam[r]) c_cur[opaque(row[r])] = cxc<R>(pl[r][1]);

    if (!ckpt) {
      // phase 1: psi and Lambda through (T_m(-B))^s together
      taylor_block<R, RPT, W, PU, 2, 1, false, LR, SPLIT>(base1, a, 0, rowb1, ok, sv, tv1, bv, ek1,
                                                      cl, ck1, m, s, (R)-1, pl, xs);
      if (a.renorm_every > 0 && n % a.renorm_every == 0) {
        CA p[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) p[r] = pl[r][0];
        renormalise<RPT, SPLIT>(p, red, a, xs);
#pragma unroll
        for (int r = 0; r < RPT; ++r) pl[r][0] = p[r];
      }
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = opaque(row[r]);
        if (own_psi[r]) c_psi[i] = pl[r][0];
        if (own_lam[r]) c_lam[i] = pl[r][1];
      }
    } else {
      // phase 1 (checkpoint variant): Lambda alone; psi_{n-1} from the segment
      CA lm[RPT][1];
#pragma unroll
      for (int r = 0; r < RPT; ++r) lm[r][0] = pl[r][1];
      C ekf[1][RPT][1];
      taylor_block<R, RPT, W, PU, 1, 1, false, LR, SPLIT>(basef, a, 0, rowbf, ok, sv, tvl, bv, ekf,
                                                      cl, ckf, m, s, (R)-1, lm, xs);
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = opaque(row[r]);
        if (own_psi[r]) c_psi[i] = cxc<double>(seg[(size_t)(n - n0) * d + i]);
        if (own_lam[r]) c_lam[i] = lm[r][0];
      }
    }

    // phase 2: auxiliary actions, G controls per pass (every Q-th pass here)
    for (int g0 = z * G; g0 < K; g0 += Q * G) {
      C ek[V2][RPT][WK];
#pragma unroll
      for (int v = 1; v < V2; ++v)
        load_E<R, RPT, WK, (PU & 4) != 0>(a, valk, g0 + v - 1, g0 + v - 1 < K, row, ok, cs, ek[v]);
      int ckl[V2][RPT][WK];
      load_colk<RPT, V2, WK, (PU & 8) != 0>(a, g0, row, ckl);
#pragma unroll
      for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int q = 0; q < WK; ++q) ek[0][r][q] = C{(R)0, (R)0};
      C yx[RPT][V2];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        // Y starts from psi_{n-1}: on the shared tail only its psi owner
        yx[r][0] = own_psi[r] ? cxc<R>(c_psi[opaque(row[r])]) : C{(R)0, (R)0};
#pragma unroll
        for (int v = 1; v < V2; ++v) yx[r][v] = C{(R)0, (R)0};
      }
      taylor_block<R, RPT, W, PU, V2, WK, true, LR, SPLIT>(base2, a, g0, rowb2, ok, sv, tv2, bv, ek,
                                                       cl, ckl, m, s, (R)1, yx, xs);
      // Re <Lambda_n|X_k>; in the rotated frame X_k = w_k X'_k, so for w_k = -i
      // Re(-i <Lambda|X'_k>) = Im <Lambda|X'_k>
      bool rot[G];
#pragma unroll
      for (int v = 0; v < G; ++v)
        rot[v] = (PU & 4) != 0 && g0 + v < K && a.ecl[g0 + v] == 0;
      double gv[G];
#pragma unroll
      for (int v = 0; v < G; ++v) gv[v] = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (ok[r]) {
          const C lc = c_cur[opaque(row[r])];
#pragma unroll
          for (int v = 0; v < G; ++v)
            gv[v] += rot[v] ? (double)lc.re * yx[r][v + 1].im - (double)lc.im * yx[r][v + 1].re
                            : (double)lc.re * yx[r][v + 1].re + (double)lc.im * yx[r][v + 1].im;
        }
      block_sum<G>(gv, red);
      if (tid == 0)
        for (int v = 0; v < G && g0 + v < K; ++v)
          a.gradp[(((size_t)b * S + h) * K + g0 + v) * N + n] = 2.0 * gv[v];
    }

    double sgr = 0.0, sgi = 0.0;  // -(w_int/(N S)) g_n for the source of psi_n
    if (a.ovt && n >= 1) {
      sgr = -cint * a.gt[((size_t)b * N + n - 1) * 2 + 0];
      sgi = -cint * a.gt[((size_t)b * N + n - 1) * 2 + 1];
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = opaque(row[r]);
      const CA ps = ok[r] ? c_psi[i] : CA{0.0, 0.0};
      pl[r][0] = own_psi[r] ? ps : CA{0.0, 0.0};
      pl[r][1] = own_lam[r] ? c_lam[i] : CA{0.0, 0.0};
      if (n >= 1 && own_lam[r] && (omega || a.ovt)) {
        const double w = omega ? cpen * omega[i] : 0.0;
        double lr = pl[r][1].re + w * ps.re;
        double li = pl[r][1].im + w * ps.im;
        if (a.ovt) {
          const double2 t = a.tgt[col0 + i];
          lr += sgr * t.x - sgi * t.y;
          li += sgr * t.y + sgi * t.x;
        }
        pl[r][1].re = lr;
        pl[r][1].im = li;
      }
    }
  }
  }

  // drift of the rebuilt initial state; in the checkpoint variant psi_0 is never
  // rebuilt, so this is only its rounding to the working precision when it was
  // stored as checkpoint 0 (zero in complex128)
  double dv[1] = {0.0};
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (own_psi[r]) {
      const double2 p0 = a.psi0[col0 + row[r]];
      const double dr = pl[r][0].re - p0.x, di = pl[r][0].im - p0.y;
      dv[0] += dr * dr + di * di;
    }
  block_sum<1>(dv, red);
  if (tid == 0 && z == 0) a.drift[(size_t)b * S + h] = sqrt(dv[0]);
}

}  // namespace hg
