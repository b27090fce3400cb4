// Dense-operator path of libhgrape: the HG cost and gradient (forward Taylor
// sweep, inverse reconstruction, co-state, auxiliary-matrix derivative,
// forbidden-level penalty, time-integrated infidelity) for operators stored as
// dense d x d matrices, as in the paper's benchmarks (Sec. IV.B), acting on a
// wide block of states (a full-basis gate problem has S = d).  Every Taylor
// term is then one dense complex contraction B . [state block], which runs on
// the matrix cores: MFMA 16x16x4 in FP32 for complex64, in FP64 for complex128.
//
// Complex arithmetic uses the real 2x2 embedding
//     a = ar + i ai  ->  [[ar, -ai], [ai, ar]],      x  ->  [xr; xi],
// so a complex d x d by d x W product is one real 2d x 2d by 2d x W product
// with the same 8 d^2 W flops.  A state block holds, per column (state h of
// group g), the 2dp real entries [Re psi; Im psi] contiguously (column-major),
// dp = d rounded up to 64 with zero rows, S rounded up to 64 with zero columns.
//
// One Taylor term (Sec. III.B, eq. eBmpsi, partial sums of App. C.2):
//     T_j = (sgn/j) B T_{j-1},   acc += T_j,
// and for the auxiliary matrix [[A, E_k],[0, A]] (Sec. III.B, eq. auxiliary
// equation) the top block of control k also takes (1/j) (E_k/s) Y_{j-1},
// Y being the bottom block (group 0).  The contraction of one term for all
// groups and all evaluations of a batch is one launch of k_term.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "hg_internal.h"

namespace hg {
namespace {

constexpr int kTPB = 256; // 4 wavefronts, 2 x 2 over the output tile
// Output tile: 32*WM rows (embedded rows) x 32*WN columns (states); each
// wavefront computes 16*WM x 16*WN as WM x WN MFMA tiles of 16 x 16.

template <typename R>
struct Mf;
template <>
struct Mf<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static constexpr int BK = 32;  // k extent of one LDS slab (128 bytes per row)
  __device__ static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in element r by lane group lg (column lane%16)
  __device__ static constexpr int row(int lg, int r) { return 4 * lg + r; }
};
template <>
struct Mf<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static constexpr int BK = 16;
  __device__ static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int lg, int r) { return lg + 4 * r; }
};

// four consecutive elements of LDS (16-byte aligned) into registers
__device__ __forceinline__ void ld4(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&o)[4]) {
  const double2 v0 = *reinterpret_cast<const double2*>(p);
  const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
  o[0] = v0.x;
  o[1] = v0.y;
  o[2] = v1.x;
  o[3] = v1.y;
}

template <typename R>
struct TermArgs {
  const R* mat;      // [B][Mp][Mp] row-major: embedded B_n = A_n / s_n
  const R* emat;     // [B][K][Mp][Mp]: embedded E_k / s_n (aux launches)
  const R* xin;      // state block read by the contraction (T_{j-1}, or P at j = 1)
  const R* accin;    // partial sum before this term
  R* tout;           // T_j
  R* accout;         // partial sum after this term
  size_t mat_b, emat_b, blk_b;  // per-evaluation strides (elements)
  int Mp, Sp, aux;   // aux: groups g >= 1 also contract E_{g-1}/s with group 0
  int n, N, rep, j;  // step (0-based), repetition (1..s), term (1..m)
  const int32_t* msch;
  const int32_t* ssch;
  R scale;           // sgn / j
};

// One Taylor term for every group of every evaluation of the batch.
// Grid: x = column tiles of 32*WN over G*Sp, y = row tiles of 32*WM over Mp, z = b.
// A workgroup whose evaluation has fewer terms (j > m_b) or repetitions
// (rep > s_b) at this step returns at once.
template <typename R, int WM, int WN>
__global__ void __launch_bounds__(kTPB) k_term(TermArgs<R> a) {
  constexpr int kBM = 32 * WM;
  constexpr int kBN = 32 * WN;
  using M = Mf<R>;
  using v4 = typename M::v4;
  constexpr int BK = M::BK;
  constexpr int VE = 16 / (int)sizeof(R);  // elements per 16-byte vector
  constexpr int RV = BK / VE;              // 16-byte vectors per slab row (8)
  constexpr int LS = BK + VE;              // padded LDS row: conflict-free 16-byte reads
  __shared__ __align__(16) R As[2][kBM * LS];
  __shared__ __align__(16) R Xs[2][kBN * LS];

  const int b = blockIdx.z;
  const int mb = a.msch[(size_t)b * a.N + a.n], sb = a.ssch[(size_t)b * a.N + a.n];
  if (a.rep > sb || a.j > mb) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const int Mp = a.Mp;
  const int c0 = blockIdx.x * kBN, i0 = blockIdx.y * kBM;
  const int g = c0 / a.Sp, cg = c0 - g * a.Sp;
  const R* matb = a.mat + (size_t)b * a.mat_b;
  const R* xb = a.xin + (size_t)b * a.blk_b;
  const int nk1 = Mp / BK;
  const int nk = (a.aux && g > 0) ? 2 * nk1 : nk1;

  constexpr int AQ = kBM * RV / kTPB;  // 16-byte A vectors per thread and slab
  constexpr int XQ = kBN * RV / kTPB;  // 16-byte X vectors per thread and slab
  v4 acc[WM][WN];
#pragma unroll
  for (int mi = 0; mi < WM; ++mi)
#pragma unroll
    for (int ni = 0; ni < WN; ++ni) acc[mi][ni] = v4{0, 0, 0, 0};

  // Iteration t loads slab t+1 into registers, computes slab t from LDS
  // buffer t&1, then stores slab t+1 to the other buffer (t = -1 only loads
  // and stores slab 0).  The staging registers are named variables: as a
  // small array the compiler placed them in spare LDS, which made every slab
  // wait for its global loads before the compute instead of after it.
  static_assert(AQ == 4 && (XQ == 2 || XQ == 4), "staging is written for 128-row tiles");
  uint4 ra0, ra1, ra2, ra3, rx0, rx1, rx2, rx3;
  for (int t = -1; t < nk; ++t) {
    const int tn = t + 1;
    if (tn < nk) {
      const bool seg1 = tn < nk1;
      const R* A = seg1 ? matb : a.emat + (size_t)b * a.emat_b + (size_t)(g - 1) * Mp * Mp;
      const R* X = xb + (size_t)(seg1 ? c0 : cg) * Mp;
      const int k0 = (seg1 ? tn : tn - nk1) * BK;
      auto ga = [&](int q) {
        const int f = tid + kTPB * q, row = f / RV, cv = f % RV;
        return *reinterpret_cast<const uint4*>(A + (size_t)(i0 + row) * Mp + k0 + cv * VE);
      };
      auto gx = [&](int q) {
        const int f = tid + kTPB * q, col = f / RV, cv = f % RV;
        return *reinterpret_cast<const uint4*>(X + (size_t)col * Mp + k0 + cv * VE);
      };
      ra0 = ga(0);
      ra1 = ga(1);
      ra2 = ga(2);
      ra3 = ga(3);
      rx0 = gx(0);
      rx1 = gx(1);
      if constexpr (XQ == 4) {
        rx2 = gx(2);
        rx3 = gx(3);
      }
    }
    if (t >= 0) {
      const R* Ab = As[t & 1];
      const R* Xb = Xs[t & 1];
      // Within a chunk of 16 k, MFMA step q takes k = kc + 4*lg + q from lane
      // group lg: each lane reads its four k of a row in one 16-byte load, and
      // A and X use the same permutation of k, so the sum over k is unchanged.
#pragma unroll
      for (int kc = 0; kc < BK; kc += 16) {
        R av[WM][4], xv[WN][4];
#pragma unroll
        for (int mi = 0; mi < WM; ++mi)
          ld4(Ab + (wm * 16 * WM + mi * 16 + lr) * LS + kc + 4 * lg, av[mi]);
#pragma unroll
        for (int ni = 0; ni < WN; ++ni)
          ld4(Xb + (wn * 16 * WN + ni * 16 + lr) * LS + kc + 4 * lg, xv[ni]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int mi = 0; mi < WM; ++mi)
#pragma unroll
            for (int ni = 0; ni < WN; ++ni)
              acc[mi][ni] = M::mma(av[mi][q], xv[ni][q], acc[mi][ni]);
      }
    }
    if (tn < nk) {
      const int buf = tn & 1;
      auto sa = [&](int q, uint4 v) {
        const int f = tid + kTPB * q, row = f / RV, cv = f % RV;
        *reinterpret_cast<uint4*>(&As[buf][row * LS + cv * VE]) = v;
      };
      auto sx = [&](int q, uint4 v) {
        const int f = tid + kTPB * q, col = f / RV, cv = f % RV;
        *reinterpret_cast<uint4*>(&Xs[buf][col * LS + cv * VE]) = v;
      };
      sa(0, ra0);
      sa(1, ra1);
      sa(2, ra2);
      sa(3, ra3);
      sx(0, rx0);
      sx(1, rx1);
      if constexpr (XQ == 4) {
        sx(2, rx2);
        sx(3, rx3);
      }
    }
    __syncthreads();
  }

  // element r of a lane's result is row M::row(lg, r), column lr, of its 16 x 16 tile
  const R* ai = a.accin + (size_t)b * a.blk_b;
  R* ao = a.accout + (size_t)b * a.blk_b;
  R* to = a.tout + (size_t)b * a.blk_b;
#pragma unroll
  for (int mi = 0; mi < WM; ++mi)
#pragma unroll
    for (int ni = 0; ni < WN; ++ni) {
      const int col = c0 + wn * 16 * WN + ni * 16 + lr;
      if constexpr (sizeof(R) == 4) {
        // complex64: the lane's four rows are contiguous, one 16-byte access each
        const size_t o = (size_t)col * Mp + i0 + wm * 16 * WM + mi * 16 + 4 * lg;
        const float4 p = *reinterpret_cast<const float4*>(ai + o);
        float4 t;
        t.x = a.scale * acc[mi][ni][0];
        t.y = a.scale * acc[mi][ni][1];
        t.z = a.scale * acc[mi][ni][2];
        t.w = a.scale * acc[mi][ni][3];
        *reinterpret_cast<float4*>(to + o) = t;
        float4 q;
        q.x = p.x + t.x;
        q.y = p.y + t.y;
        q.z = p.z + t.z;
        q.w = p.w + t.w;
        *reinterpret_cast<float4*>(ao + o) = q;
      } else {
        // complex128: element r of lane group lg is row lg + 4r.  A 4 x 4 exchange
        // across the lane groups of each column (round q: read group (lg+q)&3,
        // which sends its element lg) gives each lane rows 4lg .. 4lg+3.
        const double v0 = a.scale * acc[mi][ni][0], v1 = a.scale * acc[mi][ni][1];
        const double v2 = a.scale * acc[mi][ni][2], v3 = a.scale * acc[mi][ni][3];
        auto sel = [](int i, double x0, double x1, double x2, double x3) {
          return i == 0 ? x0 : i == 1 ? x1 : i == 2 ? x2 : x3;
        };
        double rc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          rc[q] = __shfl(sel((lg - q) & 3, v0, v1, v2, v3), lr + 16 * ((lg + q) & 3), 64);
        double t[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) t[r] = sel((r - lg) & 3, rc[0], rc[1], rc[2], rc[3]);
        const size_t o = (size_t)col * Mp + i0 + wm * 16 * WM + mi * 16 + 4 * lg;
        const double2 p0 = *reinterpret_cast<const double2*>(ai + o);
        const double2 p1 = *reinterpret_cast<const double2*>(ai + o + 2);
        *reinterpret_cast<double2*>(to + o) = double2{t[0], t[1]};
        *reinterpret_cast<double2*>(to + o + 2) = double2{t[2], t[3]};
        *reinterpret_cast<double2*>(ao + o) = double2{p0.x + t[0], p0.y + t[1]};
        *reinterpret_cast<double2*>(ao + o + 2) = double2{p1.x + t[2], p1.y + t[3]};
      }
    }
}

// theta[b][n] = dt * max_i sum_j |(H_0 + sum_k u[b][k][n] H_k)_ij|, FP64, one
// wavefront per row at a time (coalesced over j).  Row sums equal column sums
// because H_n is Hermitian (App. C).  Non-finite amplitudes give NaN.
__global__ void __launch_bounds__(256) k_dense_norms(const double2* H, const double* u, int K,
                                                     int N, int d, int dp, double dt,
                                                     double* theta) {
  __shared__ double red[4];
  const int n = blockIdx.x, b = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double* ub = u + (size_t)b * K * N;
  const size_t plane = (size_t)dp * dp;
  double mx = 0.0;
  for (int i = w; i < d; i += 4) {
    double rs = 0.0;
    for (int j = lane; j < d; j += 64) {
      const double2 v0 = H[(size_t)i * dp + j];
      double hr = v0.x, hi = v0.y;
      for (int k = 0; k < K; ++k) {
        const double c = ub[(size_t)k * N + n];
        const double2 v = H[(size_t)(k + 1) * plane + (size_t)i * dp + j];
        hr = fma(c, v.x, hr);
        hi = fma(c, v.y, hi);
      }
      rs += hypot(hr, hi);
    }
    for (int o = 32; o > 0; o >>= 1) rs += __shfl_xor(rs, o, 64);
    mx = (rs > mx || rs != rs) ? rs : mx;
  }
  if (lane == 0) red[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int q = 1; q < 4; ++q) r = (red[q] > r || red[q] != red[q]) ? red[q] : r;
    theta[(size_t)b * N + n] = dt * r;
  }
}

// Embedded A_n/s_n (and E_k/s_n) of step n for every evaluation, FP64 sums
// rounded once to the working precision.  A/s = -i (dt/s) H.
template <typename R>
__global__ void __launch_bounds__(256) k_dense_assemble(const double2* H, const double* u,
                                                        const int32_t* ssch, int K, int N, int n,
                                                        int dp, double dt, int with_e, R* mat,
                                                        R* emat, size_t mat_b, size_t emat_b) {
  const int b = blockIdx.y;
  const size_t plane = (size_t)dp * dp;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= plane) return;
  const size_t i = e / dp, jj = e % dp, Mp = 2 * (size_t)dp;
  const double c = dt / (double)ssch[(size_t)b * N + n];
  const double* ub = u + (size_t)b * K * N;
  double hr = H[e].x, hi = H[e].y;
  for (int k = 0; k < K; ++k) {
    const double uk = ub[(size_t)k * N + n];
    const double2 v = H[(size_t)(k + 1) * plane + e];
    hr = fma(uk, v.x, hr);
    hi = fma(uk, v.y, hi);
  }
  auto put = [&](R* Mx, double re, double im) {
    const R ar = (R)(c * im), ai = (R)(-c * re);  // -i c (re + i im)
    Mx[i * Mp + jj] = ar;
    Mx[i * Mp + dp + jj] = -ai;
    Mx[(dp + i) * Mp + jj] = ai;
    Mx[(dp + i) * Mp + dp + jj] = ar;
  };
  put(mat + (size_t)b * mat_b, hr, hi);
  if (with_e)
    for (int k = 0; k < K; ++k) {
      const double2 v = H[(size_t)(k + 1) * plane + e];
      put(emat + (size_t)b * emat_b + (size_t)k * Mp * Mp, v.x, v.y);
    }
}

// Group `col_off/Sp` of a state block from [B][S][d] complex128 (zero padding).
template <typename R>
__global__ void __launch_bounds__(256) k_dense_load(const double2* src, R* blk, size_t blk_b,
                                                    int S, int Sp, int d, int dp, int col_off) {
  const int b = blockIdx.y;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)Sp * dp) return;
  const int h = (int)(e / dp), i = (int)(e % dp);
  double2 v = {0.0, 0.0};
  if (h < S && i < d) v = src[((size_t)b * S + h) * d + i];
  R* c = blk + (size_t)b * blk_b + (size_t)(col_off + h) * 2 * dp;
  c[i] = (R)v.x;
  c[dp + i] = (R)v.y;
}

// dst[b][0..cnt) = src[b][0..cnt) (16-byte vectors; cnt a multiple of 16 bytes).
// With ssch: only evaluations whose step n has at least `rep` repetitions.
template <typename R>
__global__ void __launch_bounds__(256) k_dense_copy(const R* src, R* dst, size_t src_b,
                                                    size_t dst_b, size_t cnt,
                                                    const int32_t* ssch, int N, int n, int rep) {
  const int b = blockIdx.y;
  if (ssch && rep > ssch[(size_t)b * N + n]) return;
  const uint4* s = reinterpret_cast<const uint4*>(src + (size_t)b * src_b);
  uint4* t = reinterpret_cast<uint4*>(dst + (size_t)b * dst_b);
  const size_t nv = cnt * sizeof(R) / 16;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nv;
       e += (size_t)gridDim.x * blockDim.x)
    t[e] = s[e];
}

template <typename R>
__global__ void __launch_bounds__(256) k_dense_zero(R* dst, size_t dst_b, size_t cnt) {
  const int b = blockIdx.y;
  uint4* t = reinterpret_cast<uint4*>(dst + (size_t)b * dst_b);
  const size_t nv = cnt * sizeof(R) / 16;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nv;
       e += (size_t)gridDim.x * blockDim.x)
    t[e] = uint4{0u, 0u, 0u, 0u};
}

template <int NV>
__device__ __forceinline__ void block_sum256(double (&v)[NV], double* red) {
  // fixed-order reduction: wavefront butterfly, then the 4 partials in order
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[w * NV + q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = ((red[q] + red[NV + q]) + red[2 * NV + q]) + red[3 * NV + q];
}

// End of a step on group 0 of a state block, one workgroup per (state h, b):
// optional renormalisation to unit norm (complex64 reconstruction control),
// penalty <psi|Omega|psi> added to pen[b][h] (App. A, eq. c2st), overlap
// <phi_T^h|psi^h> stored as ovl (last step) and in ovt (time-integrated cost).
template <typename R>
__global__ void __launch_bounds__(256) k_dense_step_end(R* blk, size_t blk_b, int dp, int d,
                                                        int S, const double2* tgt,
                                                        const double* omega, int renorm,
                                                        double* pen, double* ovl, double* ovt,
                                                        int n, int N) {
  __shared__ double red[4 * 3];
  const int h = blockIdx.x, b = blockIdx.y;
  R* c = blk + (size_t)b * blk_b + (size_t)h * 2 * dp;
  if (renorm) {
    double nv[1] = {0.0};
    for (int i = threadIdx.x; i < d; i += blockDim.x)
      nv[0] += (double)c[i] * c[i] + (double)c[dp + i] * c[dp + i];
    block_sum256<1>(nv, red);
    const R sc = (R)(1.0 / sqrt(nv[0]));
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
      c[i] *= sc;
      c[dp + i] *= sc;
    }
  }
  if (!pen && !ovl && !ovt) return;
  double v[3] = {0.0, 0.0, 0.0};
  const double2* t = tgt + ((size_t)b * S + h) * d;
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    const double pr = c[i], pi = c[dp + i];
    if (omega) v[0] += omega[i] * (pr * pr + pi * pi);
    const double2 ti = t[i];
    v[1] += ti.x * pr + ti.y * pi;  // Re conj(phi) psi
    v[2] += ti.x * pi - ti.y * pr;  // Im conj(phi) psi
  }
  block_sum256<3>(v, red);
  if (threadIdx.x == 0) {
    if (pen && omega) pen[(size_t)b * S + h] = (n == 0 ? 0.0 : pen[(size_t)b * S + h]) + v[0];
    if (ovt) {
      ovt[(((size_t)b * S + h) * N + n) * 2 + 0] = v[1];
      ovt[(((size_t)b * S + h) * N + n) * 2 + 1] = v[2];
    }
    if (ovl && n == N - 1) {
      ovl[((size_t)b * S + h) * 2 + 0] = v[1];
      ovl[((size_t)b * S + h) * 2 + 1] = v[2];
    }
  }
}

// Cost parts of evaluation b (fixed summation order): g = (1/S) sum_h ovl,
// C1 = 1 - |g|^2, C2 = sum pen / (N S), and with ovt the step averages g_n and
// C3 = 1 - (1/N) sum_n |g_n|^2 (App. A).  res[b] = {C, C1, C2, Re g, Im g, C3}.
__global__ void __launch_bounds__(256) k_dense_finish(const double* pen, const double* ovl,
                                                      const double* ovt, double* gt,
                                                      double* res, int S, int N, double w_fid,
                                                      double w_pen, double w_int, int has_omega) {
  const int b = blockIdx.x;
  if (ovt)
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      double gr = 0.0, gi = 0.0;
      for (int h = 0; h < S; ++h) {
        gr += ovt[(((size_t)b * S + h) * N + n) * 2 + 0];
        gi += ovt[(((size_t)b * S + h) * N + n) * 2 + 1];
      }
      gt[((size_t)b * N + n) * 2 + 0] = gr / S;
      gt[((size_t)b * N + n) * 2 + 1] = gi / S;
    }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double gre = 0.0, gim = 0.0, ptot = 0.0;
  for (int h = 0; h < S; ++h) {
    gre += ovl[((size_t)b * S + h) * 2 + 0];
    gim += ovl[((size_t)b * S + h) * 2 + 1];
    ptot += pen[(size_t)b * S + h];
  }
  gre /= S;
  gim /= S;
  const double C1 = 1.0 - (gre * gre + gim * gim);
  const double C2 = has_omega ? ptot / ((double)N * S) : 0.0;
  double C3 = 0.0;
  if (ovt) {
    double q = 0.0;
    for (int n = 0; n < N; ++n) {
      const double x = gt[((size_t)b * N + n) * 2 + 0], y = gt[((size_t)b * N + n) * 2 + 1];
      q += x * x + y * y;
    }
    C3 = 1.0 - q / N;
  }
  res[(size_t)b * 8 + 0] = w_fid * C1 + (has_omega ? w_pen * C2 : 0.0) + (ovt ? w_int * C3 : 0.0);
  res[(size_t)b * 8 + 1] = C1;
  res[(size_t)b * 8 + 2] = C2;
  res[(size_t)b * 8 + 3] = gre;
  res[(size_t)b * 8 + 4] = gim;
  res[(size_t)b * 8 + 5] = C3;
}

// Co-state sources written into group 1 (Lambda) of the phase-1 block, from
// group 0 (psi) and the targets, in FP64 then rounded once:
//   turn (n = N):   Lambda_N = -(w_fid/S + cint) g phi_T + cpen Omega psi_N
//   step (n >= 1):  Lambda_n += cpen Omega psi_n - cint g_n phi_T
// with cpen = w_pen/(N S), cint = w_int/(N S) (Sec. III.A; App. A).
template <typename R>
__global__ void __launch_bounds__(256) k_dense_sources(R* blk, size_t blk_b, int dp, int d,
                                                       int S, int Sp, const double2* tgt,
                                                       const double* omega, double cpen,
                                                       const double* coef, size_t coef_b,
                                                       double coef_scale, int turn) {
  const int b = blockIdx.y;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)Sp * dp) return;
  const int h = (int)(e / dp), i = (int)(e % dp);
  R* ps = blk + (size_t)b * blk_b + (size_t)h * 2 * dp;
  R* la = blk + (size_t)b * blk_b + (size_t)(Sp + h) * 2 * dp;
  double lr = turn ? 0.0 : (double)la[i], li = turn ? 0.0 : (double)la[dp + i];
  if (h < S && i < d) {
    const double w = omega ? cpen * omega[i] : 0.0;
    lr += w * (double)ps[i];
    li += w * (double)ps[dp + i];
    if (coef) {
      const double fr = coef_scale * coef[(size_t)b * coef_b + 0];
      const double fi = coef_scale * coef[(size_t)b * coef_b + 1];
      const double2 t = tgt[((size_t)b * S + h) * d + i];
      lr += fr * t.x - fi * t.y;
      li += fr * t.y + fi * t.x;
    }
  }
  la[i] = (R)lr;
  la[dp + i] = (R)li;
}

// grad[b][k][n] = 2 sum_h Re <Lambda_n^h | X_k^h> = 2 sum over the embedded
// rows and states of Lambda * X (the real embedding turns Re conj(l) x into a
// plain dot product).  One workgroup per (k, b), fixed summation order.
template <typename R>
__global__ void __launch_bounds__(256) k_dense_grad(const R* lam, size_t lam_b, const R* wblk,
                                                    size_t w_b, int Mp, int Sp, int S, int K,
                                                    int N, int n, double* grad) {
  __shared__ double red[4];
  const int k = blockIdx.x, b = blockIdx.y;
  const R* L = lam + (size_t)b * lam_b;
  const R* X = wblk + (size_t)b * w_b + (size_t)(k + 1) * Sp * Mp;
  double v[1] = {0.0};
  const size_t cnt = (size_t)S * Mp;
  for (size_t e = threadIdx.x; e < cnt; e += blockDim.x) v[0] += (double)L[e] * (double)X[e];
  block_sum256<1>(v, red);
  if (threadIdx.x == 0) grad[((size_t)b * K + k) * N + n] = 2.0 * v[0];
}

// ||psi_0(rebuilt) - psi_0|| per state.
template <typename R>
__global__ void __launch_bounds__(256) k_dense_drift(const R* blk, size_t blk_b, int dp, int d,
                                                     int S, const double2* psi0, double* drift) {
  __shared__ double red[4];
  const int h = blockIdx.x, b = blockIdx.y;
  const R* c = blk + (size_t)b * blk_b + (size_t)h * 2 * dp;
  const double2* p0 = psi0 + ((size_t)b * S + h) * d;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < d; i += blockDim.x) {
    const double dr = (double)c[i] - p0[i].x, di = (double)c[dp + i] - p0[i].y;
    v[0] += dr * dr + di * di;
  }
  block_sum256<1>(v, red);
  if (threadIdx.x == 0) drift[(size_t)b * S + h] = sqrt(v[0]);
}

unsigned blocks_for(size_t n) { return (unsigned)std::max<size_t>(1, (n + 255) / 256); }
unsigned stride_blocks(size_t n) { return (unsigned)std::min<size_t>(1024, blocks_for(n)); }

// The four rotating state blocks of one Taylor action (P: value at the start
// of a repetition and its result; A: partial sums; T0/T1: terms).
template <typename R>
struct Rot {
  R* P;
  R* A;
  R* T[2];
  size_t stride;  // per evaluation
};

// (T_m(sgn B))^s on groups 0..G-1 of `r` for every evaluation of the batch.
template <typename R>
hipError_t taylor(const DenseShape& sh, const Rot<R>& r, int G, int aux, R sgn, int n, int smax,
                  int mmax, const R* mat, const R* emat, const int32_t* msch,
                  const int32_t* ssch, hipStream_t st) {
  const int Mp = 2 * sh.dp;
  TermArgs<R> a{};
  a.mat = mat;
  a.emat = emat;
  a.mat_b = (size_t)Mp * Mp;
  a.emat_b = (size_t)sh.K * Mp * Mp;
  a.blk_b = r.stride;
  a.Mp = Mp;
  a.Sp = sh.Sp;
  a.aux = aux;
  a.n = n;
  a.N = sh.N;
  a.msch = msch;
  a.ssch = ssch;
  // 128-row tiles; complex64 takes 128 columns when the padded state count
  // allows (a third fewer operand bytes per flop, measured +2..4%) and the
  // launch still has two workgroups per CU, else 64.  complex128 keeps 64
  // columns (at 128 its accumulators leave one wavefront per SIMD).  64 x 64
  // tiles measured far slower.
  constexpr int WM = 4;
  const size_t wg128 = (size_t)G * (sh.Sp / 128) * (Mp / (32 * WM)) * sh.B;
  const int WN = (sizeof(R) == 4 && sh.Sp % 128 == 0 && wg128 >= 2 * (size_t)sh.num_cu) ? 4 : 2;
  const dim3 grid((unsigned)(G * sh.Sp / (32 * WN)), (unsigned)(Mp / (32 * WM)), (unsigned)sh.B);
  const size_t cnt = (size_t)G * sh.Sp * Mp;
  for (int rep = 1; rep <= smax; ++rep) {
    for (int j = 1; j <= mmax; ++j) {
      a.rep = rep;
      a.j = j;
      a.xin = j == 1 ? r.P : r.T[(j - 1) & 1];
      a.accin = j == 1 ? r.P : r.A;
      a.accout = r.A;
      a.tout = r.T[j & 1];
      a.scale = sgn / (R)j;
      if constexpr (sizeof(R) == 4) {
        if (WN == 4) {
          hipLaunchKernelGGL((k_term<R, WM, 4>), grid, dim3(kTPB), 0, st, a);
          continue;
        }
      }
      hipLaunchKernelGGL((k_term<R, WM, 2>), grid, dim3(kTPB), 0, st, a);
    }
    hipLaunchKernelGGL(k_dense_copy<R>, dim3(stride_blocks(cnt), sh.B), dim3(256), 0, st,
                       (const R*)r.A, r.P, r.stride, r.stride, cnt, ssch, sh.N, n, rep);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t dense_sweep_t(const DenseOps& ops, const DenseShape& sh, const DenseBuffers& bf,
                         const SweepParams& sp, const int32_t* h_m, const int32_t* h_s,
                         hipStream_t st) {
  const int d = sh.d, dp = sh.dp, K = sh.K, N = sh.N, S = sh.S, Sp = sh.Sp, B = sh.B;
  const size_t Mp = 2 * (size_t)dp;
  const size_t grp = (size_t)Sp * Mp;  // elements of one group of one evaluation
  R* base = reinterpret_cast<R*>(bf.blocks);
  Rot<R> q{base, base + (size_t)B * 2 * grp, {base + (size_t)B * 4 * grp, base + (size_t)B * 6 * grp},
           2 * grp};
  R* wbase = base + (size_t)B * 8 * grp;
  const size_t wg = (size_t)(1 + K) * grp;
  Rot<R> wr{wbase, wbase + (size_t)B * wg, {wbase + (size_t)B * 2 * wg, wbase + (size_t)B * 3 * wg},
            wg};
  R* lkeep = wbase + (size_t)B * 4 * wg;
  R* mat = reinterpret_cast<R*>(bf.mat);
  R* emat = reinterpret_cast<R*>(bf.emat);
  const int32_t* msch = bf.m_sched;
  const int32_t* ssch = bf.s_sched;
  const double2* psi0 = reinterpret_cast<const double2*>(bf.psi0);
  const double2* tgt = reinterpret_cast<const double2*>(bf.targets);
  const unsigned eg = blocks_for((size_t)Sp * dp);
  const unsigned asm_blocks = blocks_for((size_t)dp * dp);
  auto smax = [&](int n) {
    int v = 1;
    for (int b = 0; b < B; ++b) v = std::max(v, (int)h_s[(size_t)b * N + n]);
    return v;
  };
  auto mmax = [&](int n) {
    int v = 1;
    for (int b = 0; b < B; ++b) v = std::max(v, (int)h_m[(size_t)b * N + n]);
    return v;
  };
  hipError_t e;

  // Checkpoint variant: the forward stores psi_n every C steps (whole state
  // groups); the backward re-propagates each segment forward from its
  // checkpoint, keeping its states, and propagates only Lambda backwards.
  const int C = sp.ckpt_every;
  R* ckb = reinterpret_cast<R*>(bf.ckpt);
  R* segb = reinterpret_cast<R*>(bf.segbuf);
  const size_t nseg = C > 0 ? (size_t)(N + C - 1) / C : 0;
  auto save_group = [&](const R* src, size_t src_b, R* dst, size_t dst_b) {
    hipLaunchKernelGGL(k_dense_copy<R>, dim3(stride_blocks(grp), B), dim3(256), 0, st, src, dst,
                       src_b, dst_b, grp, (const int32_t*)nullptr, N, 0, 0);
  };

  // ---- forward: psi_n = (T_m(B_n))^s psi_{n-1}, penalty and overlaps ----
  if (bf.ev[0]) (void)hipEventRecord(bf.ev[0], st);
  hipLaunchKernelGGL(k_dense_load<R>, dim3(eg, B), dim3(256), 0, st, psi0, q.P, q.stride, S, Sp,
                     d, dp, 0);
  if (C > 0) save_group(q.P, q.stride, ckb, nseg * grp);
  for (int n = 0; n < N; ++n) {
    hipLaunchKernelGGL(k_dense_assemble<R>, dim3(asm_blocks, B), dim3(256), 0, st, ops.H,
                       bf.u, ssch, K, N, n, dp, sp.dt, 0, mat, emat, Mp * Mp, (size_t)K * Mp * Mp);
    if ((e = taylor<R>(sh, q, 1, 0, (R)1, n, smax(n), mmax(n), mat, emat, msch, ssch, st)) !=
        hipSuccess)
      return e;
    const int rn = sp.renorm_every > 0 && (n + 1) % sp.renorm_every == 0;
    hipLaunchKernelGGL(k_dense_step_end<R>, dim3(S, B), dim3(256), 0, st, q.P, q.stride, dp, d,
                       S, tgt, ops.omega, rn, bf.pen, bf.ovl, bf.ovt, n, N);
    if (C > 0 && (n + 1) % C == 0 && n + 1 < N)
      save_group(q.P, q.stride, ckb + (size_t)((n + 1) / C) * grp, nseg * grp);
  }
  hipLaunchKernelGGL(k_dense_finish, dim3(B), dim3(256), 0, st, (const double*)bf.pen,
                     (const double*)bf.ovl, (const double*)bf.ovt, bf.gt, bf.res, S, N, sp.w_fid,
                     sp.w_pen, sp.w_int, ops.omega ? 1 : 0);
  // turn: Lambda_N from g (res[b][3..4]) and psi_N
  const double cpen = ops.omega ? sp.w_pen / ((double)N * S) : 0.0;
  const double cint = bf.ovt ? sp.w_int / ((double)N * S) : 0.0;
  hipLaunchKernelGGL(k_dense_sources<R>, dim3(eg, B), dim3(256), 0, st, q.P, q.stride, dp, d, S,
                     Sp, tgt, ops.omega, cpen, (const double*)(bf.res + 3), (size_t)8,
                     -(sp.w_fid / S + cint), 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (bf.ev[1]) (void)hipEventRecord(bf.ev[1], st);

  // ---- backward: n = N..1 (index n-1) ----
  // (checkpoint variant: the Lambda group alone, and a one-group rotation in
  // the phase-2 buffers for the re-propagation of a segment)
  const Rot<R> ql{q.P + grp, q.A + grp, {q.T[0] + grp, q.T[1] + grp}, q.stride};
  for (int n = N - 1; n >= 0; --n) {
    if (C > 0 && (n + 1 == N || (n + 1) % C == 0)) {
      // entering segment [n0, n]: psi_n0 from its checkpoint, then psi_n0+1..psi_n
      const int n0 = (n / C) * C;
      save_group(ckb + (size_t)(n / C) * grp, nseg * grp, wr.P, wr.stride);
      save_group(wr.P, wr.stride, segb, (size_t)C * grp);
      for (int k = n0; k < n; ++k) {
        hipLaunchKernelGGL(k_dense_assemble<R>, dim3(asm_blocks, B), dim3(256), 0, st, ops.H,
                           bf.u, ssch, K, N, k, dp, sp.dt, 0, mat, emat, Mp * Mp,
                           (size_t)K * Mp * Mp);
        if ((e = taylor<R>(sh, wr, 1, 0, (R)1, k, smax(k), mmax(k), mat, emat, msch, ssch, st)) !=
            hipSuccess)
          return e;
        const int rn = sp.renorm_every > 0 && (k + 1) % sp.renorm_every == 0;
        if (rn)
          hipLaunchKernelGGL(k_dense_step_end<R>, dim3(S, B), dim3(256), 0, st, wr.P, wr.stride,
                             dp, d, S, tgt, ops.omega, 1, (double*)nullptr, (double*)nullptr,
                             (double*)nullptr, k, N);
        save_group(wr.P, wr.stride, segb + (size_t)(k + 1 - n0) * grp, (size_t)C * grp);
      }
    }
    hipLaunchKernelGGL(k_dense_assemble<R>, dim3(asm_blocks, B), dim3(256), 0, st, ops.H,
                       bf.u, ssch, K, N, n, dp, sp.dt, K > 0 ? 1 : 0, mat, emat, Mp * Mp,
                       (size_t)K * Mp * Mp);
    // keep Lambda_n for the gradient overlaps
    hipLaunchKernelGGL(k_dense_copy<R>, dim3(stride_blocks(grp), B), dim3(256), 0, st,
                       (const R*)(q.P + grp), lkeep, q.stride, grp, grp, (const int32_t*)nullptr,
                       N, n, 0);
    // phase 1: psi_{n-1} and Lambda' through (T_m(-B_n))^s (checkpoint variant:
    // Lambda' only, psi_{n-1} from the segment's states)
    if (C > 0) {
      if ((e = taylor<R>(sh, ql, 1, 0, (R)-1, n, smax(n), mmax(n), mat, emat, msch, ssch, st)) !=
          hipSuccess)
        return e;
      save_group(segb + (size_t)(n % C) * grp, (size_t)C * grp, q.P, q.stride);
    } else if ((e = taylor<R>(sh, q, 2, 0, (R)-1, n, smax(n), mmax(n), mat, emat, msch, ssch,
                              st)) != hipSuccess) {
      return e;
    }
    if (C == 0 && sp.renorm_every > 0 && n % sp.renorm_every == 0)
      hipLaunchKernelGGL(k_dense_step_end<R>, dim3(S, B), dim3(256), 0, st, q.P, q.stride, dp, d,
                         S, tgt, ops.omega, 1, (double*)nullptr, (double*)nullptr,
                         (double*)nullptr, n, N);
    if (K > 0 && bf.grad) {
      // phase 2: (X_k; Y) = (T_m(Aux_k/s))^s (0; psi_{n-1}) for all k at once
      hipLaunchKernelGGL(k_dense_copy<R>, dim3(stride_blocks(grp), B), dim3(256), 0, st,
                         (const R*)q.P, wr.P, q.stride, wr.stride, grp, (const int32_t*)nullptr,
                         N, n, 0);
      hipLaunchKernelGGL(k_dense_zero<R>, dim3(stride_blocks((size_t)K * grp), B), dim3(256), 0,
                         st, wr.P + grp, wr.stride, (size_t)K * grp);
      if ((e = taylor<R>(sh, wr, 1 + K, 1, (R)1, n, smax(n), mmax(n), mat, emat, msch, ssch,
                         st)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(k_dense_grad<R>, dim3(K, B), dim3(256), 0, st, (const R*)lkeep, grp,
                         (const R*)wr.P, wr.stride, (int)Mp, Sp, S, K, N, n, bf.grad);
    }
    if (n >= 1 && (ops.omega || bf.ovt))
      hipLaunchKernelGGL(k_dense_sources<R>, dim3(eg, B), dim3(256), 0, st, q.P, q.stride, dp, d,
                         S, Sp, tgt, ops.omega, cpen,
                         bf.ovt ? (const double*)(bf.gt + (size_t)(n - 1) * 2) : (const double*)nullptr,
                         (size_t)2 * N, -cint, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_dense_drift<R>, dim3(S, B), dim3(256), 0, st, (const R*)q.P, q.stride, dp,
                     d, S, psi0, bf.drift);
  if (bf.ev[2]) (void)hipEventRecord(bf.ev[2], st);
  return hipGetLastError();
}

}  // namespace

size_t dense_block_elems(const DenseShape& sh) {
  const size_t grp = (size_t)sh.Sp * 2 * sh.dp;
  // phase-1 rotation (2 groups x 4), phase-2 rotation ((1+K) groups x 4), kept Lambda
  return (size_t)sh.B * grp * (8 + 4 * (size_t)(1 + sh.K) + 1);
}

hipError_t launch_dense_norms(const DenseOps& ops, int d, int dp, int K, const double* u, int nb,
                              int N, double dt, double* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_norms, dim3(N, nb), dim3(256), 0, st, ops.H, u, K, N, d, dp, dt,
                     theta);
  return hipGetLastError();
}

hipError_t launch_dense_sweep(const DenseOps& ops, const DenseShape& sh, const DenseBuffers& bf,
                              const SweepParams& sp, const int32_t* h_m, const int32_t* h_s,
                              hipStream_t st) {
  return sh.c128 ? dense_sweep_t<double>(ops, sh, bf, sp, h_m, h_s, st)
                 : dense_sweep_t<float>(ops, sh, bf, sp, h_m, h_s, st);
}

}  // namespace hg
