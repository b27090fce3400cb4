// Matrix-diagonalisation variant of the HG sweep for dense operators (App. F):
// per step the Hermitian H_n = H_0 + sum_k u_k H_k is diagonalised,
// H_n = V diag(lambda) V^H, so that
//     U_n = exp(-i dt H_n) = V diag(e^{a}) V^H,   a_i = -i dt lambda_i   (eqs. matrix dia)
//     dU_n/du_k = V (Gamma o (V^H E_k V)) V^H,     E_k = -i dt H_k        (eq. propagator der)
// with Gamma_ij the divided difference of exp at (a_i, a_j) (the e^D + E o F of
// App. F; degenerate pairs take the limit e^{a_i}, as in the oracle).  The
// sweep is the same forward-backward HG scheme as the Taylor path (Sec. III.C):
// the forward pass keeps only the current states, the backward pass rediagonalises
// H_n, rebuilds psi_{n-1} = U_n^H psi_n, carries the co-state and accumulates
//     dC/du_k[n] = 2 Re sum_h <Lambda_n^h| dU_n/du_k |psi_{n-1}^h>
//                = 2 Re sum_ab (E_k)_ab M_ab,  M = conj(V) (Gamma o P) V^T,
//     P_ij = sum_h conj(Lt_i^h) pt_j^h,  Lt = V^H Lambda_n,  pt = V^H psi_{n-1},
// so one pair of d^3 products per step serves every control (memory Theta(d^2),
// runtime O(N d^3), App. F "Scaling analysis").
//
// Eigensolver: two-sided cyclic Jacobi for complex Hermitian matrices in FP64,
// the rounds of a sweep in round-robin order (every index paired once per
// round, all pairs of a round rotated at once: A <- J^H A J with J block
// diagonal).  One launch per round updates all 2x2 blocks of A (ping-pong
// buffers, each block computing the two rotations it needs from the round's
// input) and the column pairs of V in place; after each sweep a check stops an
// evaluation once its off-diagonal part is below 1e-14 of its Frobenius norm.
// The plain complex products (V^H X, V X, X V^H) are library GEMMs (rocBLAS);
// phases, Gamma, the gradient contraction, costs and sources are kernels here.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>

#include "hg_internal.h"

namespace hg {
namespace {

constexpr int kJacobiMaxSweeps = 16;
constexpr double kJacobiTol = 1e-14;  // off(A) <= tol ||A||_F

template <typename R>
struct Cx;
template <>
struct Cx<double> {
  typedef double2 T;
};
template <>
struct Cx<float> {
  typedef float2 T;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 conjd(double2 a) { return double2{a.x, -a.y}; }

// Pair k of round r in the round-robin schedule of n2 (even) indices: player
// n2-1 stays, the others rotate.  Consecutive k give consecutive p (and
// consecutive q downwards), so a wavefront's accesses to the rows of its
// pairs are contiguous.  The pair is not sorted; either member may be the
// padding index n2-1 = d of an odd dimension.
__device__ __forceinline__ void jpair(int k, int r, int n2, int* p, int* q) {
  const int m = n2 - 1;
  *p = k == 0 ? m : (k - 1 + r) % m;
  *q = (n2 - 1 - k - 1 + r) % m;
}

// Rotation J = [[c, s], [-conj(s), c]] on coordinates (p, q) that zeroes the
// (p, q) entry of J^H A J; identity when p or q is padding or A_pq = 0.
__device__ __forceinline__ void jrot(const double2* A, int d, int p, int q, double* c, double2* s) {
  *c = 1.0;
  *s = double2{0.0, 0.0};
  if (p >= d || q >= d) return;
  const double2 z = A[p + (size_t)q * d];
  const double az = hypot(z.x, z.y);
  if (!(az > 0.0)) return;
  const double a = A[p + (size_t)p * d].x, b = A[q + (size_t)q * d].x;
  const double tau = (b - a) / (2.0 * az);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  const double cc = 1.0 / sqrt(1.0 + t * t);
  *c = cc;
  *s = double2{t * cc * z.x / az, t * cc * z.y / az};
}

// H_n into A (column-major d x d, FP64), V = I, done = 0.
__global__ void __launch_bounds__(256) k_diag_assemble(const double2* H, const double* u, int K,
                                                       int N, int n, int d, int dp, double2* A,
                                                       double2* V, int* done) {
  const int b = blockIdx.y;
  const size_t dd = (size_t)d * d;
  const double* ub = u + (size_t)b * K * N;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < dd; idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx % d), j = (int)(idx / d);
    double2 h = H[(size_t)i * dp + j];
    for (int k = 0; k < K; ++k) {
      const double c = ub[(size_t)k * N + n];
      const double2 v = H[(size_t)(k + 1) * dp * dp + (size_t)i * dp + j];
      h.x = fma(c, v.x, h.x);
      h.y = fma(c, v.y, h.y);
    }
    A[(size_t)b * dd + idx] = h;
    V[(size_t)b * dd + idx] = double2{i == j ? 1.0 : 0.0, 0.0};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) done[b] = 0;
}

// One Jacobi round for every evaluation: x in [0, nb*nb) updates the 2x2
// block (row pair x % nb, column pair x / nb) of A from Ain into Aout (the
// row pair varies fastest: column-major rows are contiguous); x in [nb*nb,
// nb*nb + d*nb) updates row i = y % d, pair y / d of V in place.
__global__ void __launch_bounds__(256) k_jac_round(const double2* Ain, double2* Aout, double2* V,
                                                   int d, int n2, int r, const int* done) {
  const int b = blockIdx.y;
  if (done[b]) return;
  const int nb = n2 / 2;
  const size_t dd = (size_t)d * d;
  const double2* A = Ain + (size_t)b * dd;
  const size_t x = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nA = (size_t)nb * nb;
  if (x < nA) {
    const int bx = (int)(x % nb), by = (int)(x / nb);
    int p, q, pp, qq;
    jpair(bx, r, n2, &p, &q);
    jpair(by, r, n2, &pp, &qq);
    double cx, cy;
    double2 sx, sy;
    jrot(A, d, p, q, &cx, &sx);
    jrot(A, d, pp, qq, &cy, &sy);
    const int ri[2] = {p, q}, ci[2] = {pp, qq};
    double2 M[2][2];
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v)
        M[u][v] = (ri[u] < d && ci[v] < d) ? A[ri[u] + (size_t)ci[v] * d] : double2{0.0, 0.0};
    // M J_y: columns (pp, qq)
    double2 T[2][2];
    for (int u = 0; u < 2; ++u) {
      const double2 m0 = M[u][0], m1 = M[u][1];
      const double2 ns = conjd(sy);
      T[u][0] = double2{cy * m0.x - (ns.x * m1.x - ns.y * m1.y), cy * m0.y - (ns.x * m1.y + ns.y * m1.x)};
      const double2 sm0 = cmul(sy, m0);
      T[u][1] = double2{sm0.x + cy * m1.x, sm0.y + cy * m1.y};
    }
    // J_x^H (M J_y): J^H = [[c, -s], [conj(s), c]]
    double2 O[2][2];
    for (int v = 0; v < 2; ++v) {
      const double2 t0 = T[0][v], t1 = T[1][v];
      const double2 st1 = cmul(sx, t1);
      O[0][v] = double2{cx * t0.x - st1.x, cx * t0.y - st1.y};
      const double2 cst0 = cmul(conjd(sx), t0);
      O[1][v] = double2{cst0.x + cx * t1.x, cst0.y + cx * t1.y};
    }
    double2* Ao = Aout + (size_t)b * dd;
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v)
        if (ri[u] < d && ci[v] < d) Ao[ri[u] + (size_t)ci[v] * d] = O[u][v];
  } else if (x < nA + (size_t)d * nb) {
    const size_t y = x - nA;
    const int i = (int)(y % d), k = (int)(y / d);
    int p, q;
    jpair(k, r, n2, &p, &q);
    if (p >= d || q >= d) return;
    double c;
    double2 s;
    jrot(A, d, p, q, &c, &s);
    double2* Vb = V + (size_t)b * dd;
    const double2 vp = Vb[i + (size_t)p * d], vq = Vb[i + (size_t)q * d];
    const double2 ns = conjd(s);
    const double2 a0 = cmul(ns, vq), a1 = cmul(s, vp);
    Vb[i + (size_t)p * d] = double2{c * vp.x - a0.x, c * vp.y - a0.y};
    Vb[i + (size_t)q * d] = double2{a1.x + c * vq.x, a1.y + c * vq.y};
  }
}

// After a sweep: off-diagonal and total Frobenius norms of A; once converged
// (or at the last sweep) the eigenvalues are its real diagonal.
__global__ void __launch_bounds__(256) k_jac_check(const double2* Acur, double* lam, int* done,
                                                   int d, double tol2, int last) {
  __shared__ double red[2][256];
  const int b = blockIdx.x;
  if (done[b]) return;
  const size_t dd = (size_t)d * d;
  const double2* A = Acur + (size_t)b * dd;
  double off = 0.0, tot = 0.0;
  for (size_t idx = threadIdx.x; idx < dd; idx += 256) {
    const double2 v = A[idx];
    const double a2 = v.x * v.x + v.y * v.y;
    tot += a2;
    if (idx % d != idx / d) off += a2;
  }
  red[0][threadIdx.x] = off;
  red[1][threadIdx.x] = tot;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  const bool conv = red[0][0] <= tol2 * red[1][0] || last;
  if (conv) {
    for (int i = threadIdx.x; i < d; i += 256) lam[(size_t)b * d + i] = A[i + (size_t)i * d].x;
    __syncthreads();
    if (threadIdx.x == 0) done[b] = 1;
  }
}

// FP64 eigenvectors into the working precision (column-major d x d).
template <typename R>
__global__ void __launch_bounds__(256) k_diag_cvt(const double2* V, typename Cx<R>::T* Vr,
                                                  size_t n) {
  const size_t b = blockIdx.y;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double2 v = V[b * n + i];
    Vr[b * n + i] = typename Cx<R>::T{(R)v.x, (R)v.y};
  }
}

// X[i][c] *= exp(sgn * (-i dt lambda_i)) for c < ncol (column-major, ld = d).
template <typename R>
__global__ void __launch_bounds__(256) k_diag_phase(typename Cx<R>::T* X, size_t xs,
                                                    const double* lam, int d, int ncol, double dt,
                                                    double sgn) {
  const int b = blockIdx.y;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < (size_t)d * ncol;
       idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx % d);
    const double ph = -sgn * dt * lam[(size_t)b * d + i];
    const double c = cos(ph), s = sin(ph);
    typename Cx<R>::T& v = X[(size_t)b * xs + idx];
    const double xr = v.x, xi = v.y;
    v.x = (R)(c * xr - s * xi);
    v.y = (R)(c * xi + s * xr);
  }
}

// Load psi0 (complex128 [S][d] = column-major d x S) into the working block.
template <typename R>
__global__ void __launch_bounds__(256) k_diag_load(const double2* src, typename Cx<R>::T* X,
                                                   size_t xs, int d, int S) {
  const int b = blockIdx.y;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < (size_t)d * S;
       idx += (size_t)gridDim.x * 256) {
    const double2 v = src[(size_t)b * d * S + idx];
    X[(size_t)b * xs + idx] = typename Cx<R>::T{(R)v.x, (R)v.y};
  }
}

// Per state column after forward step n: optional renormalisation, penalty
// sum omega |psi|^2, overlap <phi|psi> (FP64, fixed order).  One block per (h, b).
template <typename R>
__global__ void __launch_bounds__(256) k_diag_step_end(typename Cx<R>::T* X, size_t xs, int d,
                                                       int S, const double2* tgt,
                                                       const double* omega, int renorm,
                                                       double* pen, double* ovl, double* ovt,
                                                       int n, int N) {
  __shared__ double red[4][256];
  const int h = blockIdx.x, b = blockIdx.y;
  typename Cx<R>::T* x = X + (size_t)b * xs + (size_t)h * d;
  const double2* t = tgt + ((size_t)b * S + h) * d;
  double nn = 0.0;
  if (renorm) {
    for (int i = threadIdx.x; i < d; i += 256) nn += (double)x[i].x * x[i].x + (double)x[i].y * x[i].y;
    red[0][threadIdx.x] = nn;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[0][threadIdx.x] += red[0][threadIdx.x + o];
      __syncthreads();
    }
    const R sc = (R)(1.0 / sqrt(red[0][0]));
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += 256) {
      x[i].x *= sc;
      x[i].y *= sc;
    }
    __syncthreads();
  }
  double p = 0.0, orr = 0.0, oi = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double xr = x[i].x, xi = x[i].y;
    if (omega) p += omega[i] * (xr * xr + xi * xi);
    orr += t[i].x * xr + t[i].y * xi;
    oi += t[i].x * xi - t[i].y * xr;
  }
  red[1][threadIdx.x] = p;
  red[2][threadIdx.x] = orr;
  red[3][threadIdx.x] = oi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 1; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && pen) {
    pen[(size_t)b * S + h] += red[1][0];
    if (n == N - 1) {
      ovl[((size_t)b * S + h) * 2 + 0] = red[2][0];
      ovl[((size_t)b * S + h) * 2 + 1] = red[3][0];
    }
    if (ovt) {
      ovt[(((size_t)b * S + h) * N + n) * 2 + 0] = red[2][0];
      ovt[(((size_t)b * S + h) * N + n) * 2 + 1] = red[3][0];
    }
  }
}

__global__ void __launch_bounds__(256) k_diag_zero(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    p[i] = 0.0;
}

// Cost parts from the FP64 partials (C1 from g, C2, C3 from the per-step overlaps).
__global__ void __launch_bounds__(256) k_diag_finish(const double* pen, const double* ovl,
                                                     const double* ovt, double* gt, double* res,
                                                     int S, int N, double w_fid, double w_pen,
                                                     double w_int, int has_omega) {
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

// Co-state sources: turn (init = 1) sets Lambda = f g phi + cpen Omega psi;
// otherwise Lambda += cint_g phi + cpen Omega psi, with the coefficient of phi
// f * gsrc (gsrc: g of the turn, or g_n of the time-integrated term).
template <typename R>
__global__ void __launch_bounds__(256) k_diag_sources(const typename Cx<R>::T* X, typename Cx<R>::T* L,
                                                      size_t xs, int d, int S, const double2* tgt,
                                                      const double* omega, double cpen,
                                                      const double* gsrc, size_t gsrc_b, double f,
                                                      int init) {
  const int b = blockIdx.y;
  double gr = 0.0, gi = 0.0;
  if (gsrc) {
    gr = f * gsrc[(size_t)b * gsrc_b + 0];
    gi = f * gsrc[(size_t)b * gsrc_b + 1];
  }
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < (size_t)d * S;
       idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx % d);
    const double2 t = tgt[(size_t)b * d * S + idx];
    const typename Cx<R>::T x = X[(size_t)b * xs + idx];
    const double w = omega ? cpen * omega[i] : 0.0;
    double lr = gr * t.x - gi * t.y + w * (double)x.x;
    double li = gr * t.y + gi * t.x + w * (double)x.y;
    typename Cx<R>::T& l = L[(size_t)b * xs + idx];
    if (!init) {
      lr += (double)l.x;
      li += (double)l.y;
    }
    l.x = (R)lr;
    l.y = (R)li;
  }
}

// G = Gamma o PT in place (PT = pt Lt^H, column-major d x d):
// Gamma_ij = exp(-i dt (l_i + l_j)/2) sinc(dt (l_i - l_j)/2), the divided
// difference of exp at a_i = -i dt l_i, a_j (symmetric; exact limit at a_i = a_j).
template <typename R>
__global__ void __launch_bounds__(256) k_diag_gamma(typename Cx<R>::T* PT, size_t ps,
                                                    const double* lam, int d, double dt) {
  const int b = blockIdx.y;
  const double* l = lam + (size_t)b * d;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < (size_t)d * d;
       idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx % d), j = (int)(idx / d);
    const double m = -0.5 * dt * (l[i] + l[j]);
    const double x = 0.5 * dt * (l[i] - l[j]);
    const double sc = fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x;
    const double gr = cos(m) * sc, gi = sin(m) * sc;
    typename Cx<R>::T& v = PT[(size_t)b * ps + idx];
    const double vr = v.x, vi = v.y;
    v.x = (R)(gr * vr - gi * vi);
    v.y = (R)(gr * vi + gi * vr);
  }
}

// grad[b][k][n] = 2 Re tr(E_k Q) with E_k = -i dt H_k, Q = M^T column-major:
// tr(E Q) = sum over the row-major entries of H_k times the same linear
// index of Q, so grad = 2 dt Im(sum_L H_k[L] Q[L]).  One block per (k, b).
template <typename R>
__global__ void __launch_bounds__(256) k_diag_grad(const double2* H, const typename Cx<R>::T* Q,
                                                   size_t qs, int d, int dp, int K, int N, int n,
                                                   double dt, double* grad) {
  __shared__ double red[256];
  const int k = blockIdx.x, b = blockIdx.y;
  const double2* Hk = H + (size_t)(k + 1) * dp * dp;
  const typename Cx<R>::T* q = Q + (size_t)b * qs;
  double im = 0.0;
  for (size_t idx = threadIdx.x; idx < (size_t)d * d; idx += 256) {
    const int a = (int)(idx / d), c = (int)(idx % d);   // H[a][c] <-> Q(c, a)
    const double2 h = Hk[(size_t)a * dp + c];
    const typename Cx<R>::T v = q[idx];
    im += h.x * (double)v.y + h.y * (double)v.x;
  }
  red[threadIdx.x] = im;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[((size_t)b * K + k) * N + n] = 2.0 * dt * red[0];
}

// drift = max over the columns is taken on the host; here ||psi_0(rebuilt) - psi_0|| per column
template <typename R>
__global__ void __launch_bounds__(256) k_diag_drift(const typename Cx<R>::T* X, size_t xs, int d,
                                                    int S, const double2* psi0, double* drift) {
  __shared__ double red[256];
  const int h = blockIdx.x, b = blockIdx.y;
  double s = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const typename Cx<R>::T x = X[(size_t)b * xs + (size_t)h * d + i];
    const double2 p = psi0[((size_t)b * S + h) * d + i];
    const double dr = (double)x.x - p.x, di = (double)x.y - p.y;
    s += dr * dr + di * di;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) drift[(size_t)b * S + h] = sqrt(red[0]);
}

unsigned nblk(size_t n) { return (unsigned)std::min<size_t>(4096, (n + 255) / 256); }

// rocBLAS handle of the calling thread for device `dev` (created on first use).
struct Handles {
  std::map<int, rocblas_handle> h;
  ~Handles() {
    for (auto& kv : h) (void)rocblas_destroy_handle(kv.second);
  }
};
thread_local Handles t_blas;

rocblas_handle blas_for(int dev) {
  auto it = t_blas.h.find(dev);
  if (it != t_blas.h.end()) return it->second;
  rocblas_handle hd = nullptr;
  if (rocblas_create_handle(&hd) != rocblas_status_success) return nullptr;
  t_blas.h[dev] = hd;
  return hd;
}

// C = op(A) op(B) for every evaluation (column-major, strided batch).
template <typename R>
rocblas_status gemm(rocblas_handle hd, rocblas_operation ta, rocblas_operation tb, int m, int n,
                    int k, const typename Cx<R>::T* A, int lda, size_t sa,
                    const typename Cx<R>::T* Bm, int ldb, size_t sb, typename Cx<R>::T* C, int ldc,
                    size_t sc, int batch) {
  if constexpr (sizeof(R) == 8) {
    const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0};
    return rocblas_zgemm_strided_batched(
        hd, ta, tb, m, n, k, &one, reinterpret_cast<const rocblas_double_complex*>(A), lda,
        (rocblas_stride)sa, reinterpret_cast<const rocblas_double_complex*>(Bm), ldb,
        (rocblas_stride)sb, &zero, reinterpret_cast<rocblas_double_complex*>(C), ldc,
        (rocblas_stride)sc, batch);
  } else {
    const rocblas_float_complex one{1.0f, 0.0f}, zero{0.0f, 0.0f};
    return rocblas_cgemm_strided_batched(
        hd, ta, tb, m, n, k, &one, reinterpret_cast<const rocblas_float_complex*>(A), lda,
        (rocblas_stride)sa, reinterpret_cast<const rocblas_float_complex*>(Bm), ldb,
        (rocblas_stride)sb, &zero, reinterpret_cast<rocblas_float_complex*>(C), ldc,
        (rocblas_stride)sc, batch);
  }
}

#define HG_BLAS(call)                                               \
  do {                                                              \
    if ((call) != rocblas_status_success) return hipErrorUnknown;   \
  } while (0)

struct DiagMem {
  double2 *A0, *A1, *V;
  double* lam;
  int* done;
  void* Vr;    // working-precision eigenvectors (complex64 only)
  void* X;     // [psi | Lambda] block, d x 2S
  void* Y;     // its eigenbasis copy, d x 2S
  void* PT;    // d x d
  void* Z;     // d x d
  double *pen, *ovl, *ovt, *gt, *drift, *res;
  size_t dd, xs;
};

// Diagonalise H_n for every evaluation: eigenvalues into lam, eigenvectors V.
// After each sweep the host reads the convergence flags (one small copy) and
// stops launching rounds once every evaluation has converged.
hipError_t diagonalise(const DenseOps& ops, const DenseShape& sh, const DiagMem& m,
                       const double* u, int n, int* h_done, hipStream_t st) {
  const int d = sh.d, B = sh.B;
  const int n2 = d + (d & 1);
  hipLaunchKernelGGL(k_diag_assemble, dim3(nblk(m.dd), B), dim3(256), 0, st, ops.H, u, sh.K,
                     sh.N, n, d, sh.dp, m.A0, m.V, m.done);
  double2* cur = m.A0;
  double2* nxt = m.A1;
  const size_t nb = (size_t)n2 / 2;
  const unsigned gx = (unsigned)((nb * nb + (size_t)d * nb + 255) / 256);
  for (int sw = 0; sw < kJacobiMaxSweeps; ++sw) {
    for (int r = 0; r < n2 - 1; ++r) {
      hipLaunchKernelGGL(k_jac_round, dim3(gx, B), dim3(256), 0, st, (const double2*)cur, nxt,
                         m.V, d, n2, r, (const int*)m.done);
      std::swap(cur, nxt);
    }
    hipLaunchKernelGGL(k_jac_check, dim3(B), dim3(256), 0, st, (const double2*)cur, m.lam, m.done,
                       d, kJacobiTol * kJacobiTol, sw == kJacobiMaxSweeps - 1 ? 1 : 0);
    hipError_t e = hipMemcpyAsync(h_done, m.done, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    bool all = true;
    for (int b = 0; b < B; ++b) all = all && h_done[b] != 0;
    if (all) break;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t diag_sweep_t(int dev, const DenseOps& ops, const DenseShape& sh, const DiagBuffers& bf,
                        const SweepParams& sp, hipStream_t st) {
  using T = typename Cx<R>::T;
  const int d = sh.d, K = sh.K, N = sh.N, S = sh.S, B = sh.B, dp = sh.dp;
  rocblas_handle hd = blas_for(dev);
  if (!hd) return hipErrorUnknown;
  HG_BLAS(rocblas_set_stream(hd, st));
  DiagMem m{};
  m.dd = (size_t)d * d;
  m.xs = (size_t)d * 2 * S;
  char* w = reinterpret_cast<char*>(bf.work);
  auto take = [&](size_t bytes) {
    char* p = w;
    w += (bytes + 255) & ~(size_t)255;
    return p;
  };
  m.A0 = (double2*)take((size_t)B * m.dd * 16);
  m.A1 = (double2*)take((size_t)B * m.dd * 16);
  m.V = (double2*)take((size_t)B * m.dd * 16);
  m.lam = (double*)take((size_t)B * d * 8);
  m.done = (int*)take((size_t)B * 4);
  m.Vr = sizeof(R) == 4 ? take((size_t)B * m.dd * sizeof(T)) : nullptr;
  m.X = take((size_t)B * m.xs * sizeof(T));
  m.Y = take((size_t)B * m.xs * sizeof(T));
  m.PT = take((size_t)B * m.dd * sizeof(T));
  m.Z = take((size_t)B * m.dd * sizeof(T));
  const T* V = sizeof(R) == 4 ? (const T*)m.Vr : (const T*)m.V;
  T* X = (T*)m.X;           // columns 0..S-1: psi, S..2S-1: Lambda
  T* Xl = X + (size_t)d * S;
  T* Y = (T*)m.Y;
  T* Yl = Y + (size_t)d * S;
  T* PT = (T*)m.PT;
  T* Z = (T*)m.Z;
  const double2* psi0 = reinterpret_cast<const double2*>(bf.psi0);
  const double2* tgt = reinterpret_cast<const double2*>(bf.targets);
  const unsigned gx = nblk((size_t)d * 2 * S);
  auto eig = [&](int n) -> hipError_t {
    hipError_t e = diagonalise(ops, sh, m, bf.u, n, bf.h_done, st);
    if (e != hipSuccess) return e;
    if (sizeof(R) == 4)
      hipLaunchKernelGGL(k_diag_cvt<R>, dim3(nblk(m.dd), B), dim3(256), 0, st,
                         (const double2*)m.V, (T*)m.Vr, m.dd);
    return hipGetLastError();
  };
  const auto N_ = rocblas_operation_none, C_ = rocblas_operation_conjugate_transpose;

  // ---- forward ----
  if (bf.ev[0]) (void)hipEventRecord(bf.ev[0], st);
  hipLaunchKernelGGL(k_diag_zero, dim3(1), dim3(256), 0, st, bf.pen, (size_t)B * S);
  hipLaunchKernelGGL(k_diag_load<R>, dim3(gx, B), dim3(256), 0, st, psi0, X, m.xs, d, S);
  hipError_t e;
  for (int n = 0; n < N; ++n) {
    if ((e = eig(n)) != hipSuccess) return e;
    // psi_n = V e^{a} V^H psi_{n-1}
    HG_BLAS(gemm<R>(hd, C_, N_, d, S, d, V, d, m.dd, X, d, m.xs, Y, d, m.xs, B));
    hipLaunchKernelGGL(k_diag_phase<R>, dim3(gx, B), dim3(256), 0, st, Y, m.xs,
                       (const double*)m.lam, d, S, sp.dt, 1.0);
    HG_BLAS(gemm<R>(hd, N_, N_, d, S, d, V, d, m.dd, Y, d, m.xs, X, d, m.xs, B));
    const int rn = sp.renorm_every > 0 && (n + 1) % sp.renorm_every == 0;
    hipLaunchKernelGGL(k_diag_step_end<R>, dim3(S, B), dim3(256), 0, st, X, m.xs, d, S, tgt,
                       ops.omega, rn, bf.pen, bf.ovl, bf.ovt, n, N);
  }
  hipLaunchKernelGGL(k_diag_finish, dim3(B), dim3(256), 0, st, (const double*)bf.pen,
                     (const double*)bf.ovl, (const double*)bf.ovt, bf.gt, bf.res, S, N, sp.w_fid,
                     sp.w_pen, sp.w_int, ops.omega ? 1 : 0);
  const double cpen = ops.omega ? sp.w_pen / ((double)N * S) : 0.0;
  const double cint = bf.ovt ? sp.w_int / ((double)N * S) : 0.0;
  // turn: Lambda_N = -(w_fid/S + cint) g phi + cpen Omega psi_N
  hipLaunchKernelGGL(k_diag_sources<R>, dim3(nblk((size_t)d * S), B), dim3(256), 0, st,
                     (const T*)X, Xl, m.xs, d, S, tgt, ops.omega, cpen,
                     (const double*)(bf.res + 3), (size_t)8, -(sp.w_fid / S + cint), 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (bf.ev[1]) (void)hipEventRecord(bf.ev[1], st);

  // ---- backward: n = N..1 (index n-1) ----
  for (int n = N - 1; n >= 0; --n) {
    if ((e = eig(n)) != hipSuccess) return e;
    // [pt | Lt] = V^H [psi_n | Lambda_n]; pt <- e^{-a} pt (psi_{n-1} in the eigenbasis)
    HG_BLAS(gemm<R>(hd, C_, N_, d, 2 * S, d, V, d, m.dd, X, d, m.xs, Y, d, m.xs, B));
    hipLaunchKernelGGL(k_diag_phase<R>, dim3(gx, B), dim3(256), 0, st, Y, m.xs,
                       (const double*)m.lam, d, S, sp.dt, -1.0);
    if (K > 0 && bf.grad) {
      // PT = pt Lt^H, G = Gamma o PT, Q = V G V^H, grad_k = 2 Re tr(E_k Q)
      HG_BLAS(gemm<R>(hd, N_, C_, d, d, S, Y, d, m.xs, Yl, d, m.xs, PT, d, m.dd, B));
      hipLaunchKernelGGL(k_diag_gamma<R>, dim3(nblk(m.dd), B), dim3(256), 0, st, PT, m.dd,
                         (const double*)m.lam, d, sp.dt);
      HG_BLAS(gemm<R>(hd, N_, N_, d, d, d, V, d, m.dd, PT, d, m.dd, Z, d, m.dd, B));
      HG_BLAS(gemm<R>(hd, N_, C_, d, d, d, Z, d, m.dd, V, d, m.dd, PT, d, m.dd, B));
      hipLaunchKernelGGL(k_diag_grad<R>, dim3(K, B), dim3(256), 0, st, ops.H, (const T*)PT, m.dd,
                         d, dp, K, N, n, sp.dt, bf.grad);
    }
    // Lambda' in the eigenbasis: e^{-a} Lt; back to the standard basis with psi_{n-1}
    hipLaunchKernelGGL(k_diag_phase<R>, dim3(gx, B), dim3(256), 0, st, Yl, m.xs,
                       (const double*)m.lam, d, S, sp.dt, -1.0);
    HG_BLAS(gemm<R>(hd, N_, N_, d, 2 * S, d, V, d, m.dd, Y, d, m.xs, X, d, m.xs, B));
    if (sp.renorm_every > 0 && n % sp.renorm_every == 0)
      hipLaunchKernelGGL(k_diag_step_end<R>, dim3(S, B), dim3(256), 0, st, X, m.xs, d, S, tgt,
                         ops.omega, 1, (double*)nullptr, (double*)nullptr, (double*)nullptr, n, N);
    if (n >= 1 && (ops.omega || bf.ovt))
      hipLaunchKernelGGL(k_diag_sources<R>, dim3(nblk((size_t)d * S), B), dim3(256), 0, st,
                         (const T*)X, Xl, m.xs, d, S, tgt, ops.omega, cpen,
                         bf.ovt ? (const double*)(bf.gt + (size_t)(n - 1) * 2) : (const double*)nullptr,
                         (size_t)2 * N, -cint, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_diag_drift<R>, dim3(S, B), dim3(256), 0, st, (const T*)X, m.xs, d, S,
                     psi0, bf.drift);
  if (bf.ev[2]) (void)hipEventRecord(bf.ev[2], st);
  return hipGetLastError();
}

}  // namespace

size_t diag_work_bytes(const DenseShape& sh) {
  const size_t d = (size_t)sh.d, B = (size_t)sh.B, S = (size_t)sh.S;
  const size_t cs = sh.c128 ? 16 : 8;
  auto a = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return a(B * d * d * 16) * 3 + a(B * d * 8) + a(B * 4) + (sh.c128 ? 0 : a(B * d * d * cs)) +
         2 * a(B * d * 2 * S * cs) + 2 * a(B * d * d * cs);
}

hipError_t launch_diag_sweep(int dev, const DenseOps& ops, const DenseShape& sh,
                             const DiagBuffers& bf, const SweepParams& sp, hipStream_t st) {
  return sh.c128 ? diag_sweep_t<double>(dev, ops, sh, bf, sp, st)
                 : diag_sweep_t<float>(dev, ops, sh, bf, sp, st);
}

}  // namespace hg
