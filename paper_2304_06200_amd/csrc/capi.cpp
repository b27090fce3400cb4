// C ABI of libhgrape: validation, operator conversion (CSR -> DIA on the
// device), evaluation orchestration (norms -> host planner -> sweeps).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "hg_internal.h"

namespace hg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

hg_status fail(hg_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

hg_status hip_fail(hipError_t e, const char* what) {
  return fail(HG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HG_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

struct Entry {
  int64_t col;
  double re, im;
};

// Validated, duplicate-summed rows of one CSR operator (explicit zeros dropped).
hg_status read_csr(const hg_csr* m, int64_t dim, const char* name,
                   std::vector<std::vector<Entry>>* rows) {
  if (!m || m->n != dim || !m->indptr) return fail(HG_ERR_INVALID_ARG, std::string(name) + ": shape or indptr");
  if (m->indptr[0] != 0) return fail(HG_ERR_INVALID_ARG, std::string(name) + ": indptr[0] != 0");
  for (int64_t i = 0; i < dim; ++i)
    if (m->indptr[i + 1] < m->indptr[i])
      return fail(HG_ERR_INVALID_ARG, std::string(name) + ": indptr not monotone");
  const int64_t nnz = m->indptr[dim];
  if (nnz > 0 && (!m->indices || !m->values))
    return fail(HG_ERR_INVALID_ARG, std::string(name) + ": missing indices/values");
  rows->assign(dim, {});
  for (int64_t i = 0; i < dim; ++i) {
    std::map<int64_t, std::pair<double, double>> acc;
    for (int64_t p = m->indptr[i]; p < m->indptr[i + 1]; ++p) {
      const int64_t j = m->indices[p];
      if (j < 0 || j >= dim) return fail(HG_ERR_INVALID_ARG, std::string(name) + ": column out of range");
      const double re = m->values[2 * p], im = m->values[2 * p + 1];
      if (!std::isfinite(re) || !std::isfinite(im))
        return fail(HG_ERR_NONFINITE, std::string(name) + ": non-finite value");
      auto& a = acc[j];
      a.first += re;
      a.second += im;
    }
    for (auto& kv : acc)
      if (kv.second.first != 0.0 || kv.second.second != 0.0)
        (*rows)[i].push_back({kv.first, kv.second.first, kv.second.second});
  }
  return HG_OK;
}

hg_status check_hermitian(const std::vector<std::vector<Entry>>& rows, const char* name) {
  double amax = 0.0;
  for (auto& r : rows)
    for (auto& e : r) amax = std::max(amax, std::hypot(e.re, e.im));
  const double tol = 1e-12 * (amax > 0 ? amax : 1.0);
  auto find = [&](int64_t i, int64_t j, double* re, double* im) {
    const auto& r = rows[i];
    auto it = std::lower_bound(r.begin(), r.end(), j,
                               [](const Entry& e, int64_t c) { return e.col < c; });
    if (it != r.end() && it->col == j) {
      *re = it->re;
      *im = it->im;
    } else {
      *re = 0.0;
      *im = 0.0;
    }
  };
  for (int64_t i = 0; i < (int64_t)rows.size(); ++i)
    for (auto& e : rows[i]) {
      double tr, ti;
      find(e.col, i, &tr, &ti);
      if (std::fabs(e.re - tr) > tol || std::fabs(e.im + ti) > tol)
        return fail(HG_ERR_NOT_HERMITIAN, std::string(name) + " is not Hermitian at (" +
                                              std::to_string(i) + "," + std::to_string(e.col) + ")");
    }
  return HG_OK;
}

}  // namespace
}  // namespace hg

using namespace hg;

// The C entry points below never let an exception out: a failed host
// allocation becomes OUT_OF_MEMORY, anything else DEVICE.
template <typename F>
hg_status guarded(const char* what, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(HG_ERR_OUT_OF_MEMORY, std::string(what) + ": host allocation failed");
  } catch (const std::exception& e) {
    return fail(HG_ERR_DEVICE, std::string(what) + ": " + e.what());
  } catch (...) {
    return fail(HG_ERR_DEVICE, std::string(what) + ": unexpected exception");
  }
}


namespace hg {
namespace {

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Chooses the column split of a banded problem (see Split): the smallest halo
// width h for which the offsets larger than h have a common block length L
// with dim % L == 0 and no entry at an offset of at most h crosses a block,
// then the fewest parts P whose local problem the kernels take in both
// precisions.  Fills sp (without device arrays) or returns false with why.
bool plan_split(const std::vector<std::vector<std::vector<Entry>>>& ops, int64_t dim,
                const DevOps& g, int K, size_t lds, int num_cu, Split* sp, std::string* why) {
  std::set<int64_t> mags;
  mags.insert(0);
  for (int e = 0; e < g.W; ++e)
    if (g.off[e] != 0) mags.insert(std::llabs((int64_t)g.off[e]));
  for (int64_t hh : mags) {
    int64_t Lg = 0;
    for (int e = 0; e < g.W; ++e)
      if (std::llabs((int64_t)g.off[e]) > hh) Lg = gcd64(Lg, std::llabs((int64_t)g.off[e]));
    const int64_t L = Lg ? Lg : dim;
    if (L < 2 || dim % L != 0 || L <= 2 * hh) continue;
    bool inside = true;
    for (size_t o = 0; o < ops.size() && inside; ++o)
      for (int64_t i = 0; i < dim && inside; ++i)
        for (auto& en : ops[o][i])
          if (en.col != i && std::llabs(en.col - i) <= hh && en.col / L != i / L) {
            inside = false;
            break;
          }
    if (!inside) continue;
    const int64_t T = dim / L;
    for (int P = 2; P <= kMaxParts; ++P) {
      if (L / P < std::max<int64_t>(hh, 1)) break;
      Split c;
      c.P = P;
      c.L = (int)L;
      c.T = (int)T;
      c.h = (int)hh;
      int wmax = 0, c0 = 0;
      for (int q = 0; q < P; ++q) {
        c.w[q] = (int)(L / P + (q < L % P ? 1 : 0));
        c.c0[q] = c0;
        c0 += c.w[q];
        wmax = std::max(wmax, c.w[q]);
      }
      c.seg = wmax + 2 * (int)hh;
      if ((int64_t)T * c.seg > (int64_t)kMaxThreads * kMaxRows) continue;
      c.d_loc = (int)T * c.seg;
      auto local = [&](int o) {
        return std::llabs((int64_t)o) <= hh ? o : (int)((int64_t)o / L) * c.seg;
      };
      c.ops.W = g.W;
      c.ops.npure = g.npure;
      c.ops.ereal = g.ereal;
      for (int k = 0; k < K; ++k) c.ops.ecl[k] = g.ecl[k];
      c.ops.halo = 0;
      for (int e = 0; e < g.W; ++e) {
        c.ops.off[e] = local(g.off[e]);
        c.ops.halo = std::max(c.ops.halo, std::abs(c.ops.off[e]));
      }
      for (int k = 0; k < K; ++k) {
        c.ops.WK[k] = g.WK[k];
        for (int q = 0; q < g.WK[k]; ++q) c.ops.offk[k][q] = local(g.offk[k][q]);
      }
      SweepShape sh{};
      std::string w1, w2;
      if (split_supported(c, K, true, lds, num_cu, &sh, &w1) &&
          split_supported(c, K, false, lds, num_cu, &sh, &w2)) {
        *sp = c;
        return true;
      }
    }
  }
  *why = "no split of the rows over up to " + std::to_string(kMaxParts) +
         " workgroups fits: the union offsets do not separate into a block length L (dim % L "
         "== 0) and short offsets that stay inside their block";
  return false;
}

}  // namespace
}  // namespace hg

hg_problem::~hg_problem() {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ops.vals) (void)hipFree(ops.vals);
  if (ops.valk) (void)hipFree(ops.valk);
  if (ops.omega) (void)hipFree(ops.omega);
  if (ops.cols) (void)hipFree(ops.cols);
  if (ops.colk) (void)hipFree(ops.colk);
  if (dops.H) (void)hipFree(dops.H);
  if (split.ops.vals) (void)hipFree(split.ops.vals);
  if (split.ops.valk) (void)hipFree(split.ops.valk);
  if (split.ops.omega) (void)hipFree(split.ops.omega);
}

extern "C" {

const char* hg_status_string(hg_status s) {
  switch (s) {
    case HG_OK: return "ok";
    case HG_ERR_INVALID_ARG: return "invalid argument";
    case HG_ERR_NOT_HERMITIAN: return "operator not Hermitian";
    case HG_ERR_NONFINITE: return "non-finite input";
    case HG_ERR_TOLERANCE_UNREACHABLE: return "tolerance unreachable";
    case HG_ERR_OUT_OF_MEMORY: return "out of memory";
    case HG_ERR_DEVICE: return "device error";
    case HG_ERR_BUSY: return "busy";
    case HG_ERR_CANCELLED: return "cancelled";
    case HG_ERR_UNSUPPORTED: return "unsupported shape";
  }
  return "unknown status";
}

const char* hg_last_error(void) { return g_last_error.c_str(); }

int32_t hg_version(void) { return 100; }

hg_status hg_create(int device_ordinal, hg_ctx** out) {
  if (!out) return fail(HG_ERR_INVALID_ARG, "out is NULL");
  int n = 0;
  HG_HIP(hipGetDeviceCount(&n));
  if (device_ordinal < 0 || device_ordinal >= n)
    return fail(HG_ERR_INVALID_ARG, "device ordinal out of range");
  HG_HIP(hipSetDevice(device_ordinal));
  auto c = std::make_unique<hg_ctx>();
  c->device = device_ordinal;
  int v = 0;
  HG_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device_ordinal));
  c->num_cu = v;
  HG_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device_ordinal));
  c->lds_per_block = (size_t)v;
  // evaluation workspaces come from the device's default pool (hipMallocAsync):
  // keep freed blocks in the pool instead of returning them at every sync
  hipMemPool_t pool;
  HG_HIP(hipDeviceGetDefaultMemPool(&pool, device_ordinal));
  uint64_t keep = UINT64_MAX;
  HG_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  // device address of hg_eval_noalloc's scratch array on this device
  hg_status st = noalloc_setup(device_ordinal);
  if (st != HG_OK) return st;
  *out = c.release();
  return HG_OK;
}

hg_status hg_destroy(hg_ctx* ctx) {
  delete ctx;
  return HG_OK;
}

// Control classes: every entry of H_k real (ecl 0: E_k = -i (dt/s) H_k purely
// imaginary) or every entry purely imaginary (ecl 1: E_k real); ereal when
// all controls are one or the other (the rotated frame of the auxiliary
// vectors then applies).
static void classify_controls(const std::vector<std::vector<std::vector<Entry>>>& ops, int64_t dim,
                              int K, DevOps* d) {
  d->ereal = K > 0;
  for (int k = 0; k < K; ++k) {
    bool re_only = true, im_only = true;
    for (int64_t i = 0; i < dim; ++i)
      for (auto& en : ops[k + 1][i]) {
        if (en.im != 0.0) re_only = false;
        if (en.re != 0.0) im_only = false;
      }
    d->ecl[k] = re_only ? 0 : 1;
    if (!re_only && !im_only) d->ereal = false;
  }
}

// Row-indexed (ELL) storage for patterns that are not a few diagonals (a
// qubit register's bit flips, a random sparse coupling): per row the union
// columns in slots, slot 0 the main diagonal (an all-zero stand-in when the
// main diagonal is complex somewhere, which then takes an ordinary slot), and
// per control its own columns (at most 2 per row).  Held by one workgroup per
// column (no split).
static hg_status create_ell(hg_ctx* ctx, int64_t dim, int K,
                            const std::vector<std::vector<std::vector<Entry>>>& ops,
                            const double* omega_diag, bool diag_complex, int64_t sigma,
                            int64_t nnz, const std::vector<int64_t>& nnz_ctrl, hg_problem** out) {
  std::vector<std::vector<int64_t>> rc((size_t)dim);
  int W = 1;
  std::vector<int> ek((size_t)std::max(K, 1), 0);
  for (int64_t i = 0; i < dim; ++i) {
    std::set<int64_t> cs;
    for (int o = 0; o <= K; ++o)
      for (auto& e : ops[o][i]) cs.insert(e.col);
    std::vector<int64_t>& v = rc[(size_t)i];
    v.push_back(i);
    for (int64_t c : cs)
      if (c != i || diag_complex) v.push_back(c);
    W = std::max(W, (int)v.size());
    for (int k = 0; k < K; ++k) ek[k] = std::max(ek[k], (int)ops[k + 1][i].size());
  }
  if (W > kMaxDiagKernels)
    return fail(HG_ERR_UNSUPPORTED, "a row has " + std::to_string(W) + " stored entries (counting a "
                                    "slot for the main diagonal); the sweep kernels take at most 13 "
                                    "(hg_problem_create_dense stores operators densely)");
  for (int k = 0; k < K; ++k)
    if (ek[k] > 2)
      return fail(HG_ERR_UNSUPPORTED, "control " + std::to_string(k + 1) + " has " +
                                          std::to_string(ek[k]) + " entries in a row; row-indexed "
                                          "storage takes at most 2 (dense storage takes any)");
  auto p = std::make_unique<hg_problem>();
  p->ctx = ctx;
  p->dim = dim;
  p->n_ctrl = K;
  p->sigma = (int32_t)std::max<int64_t>(sigma, 1);
  p->nnz = nnz;
  p->nnz_ctrl = nnz_ctrl;
  DevOps& d = p->ops;
  d.ell = true;
  d.W = W;
  d.npure = 1;
  d.halo = 0;
  classify_controls(ops, dim, K, &d);
  for (int k = 0; k < K; ++k) d.WK[k] = ek[k];
  const size_t D = (size_t)dim;
  std::vector<int32_t> hc((size_t)W * D), hck((size_t)std::max(K, 1) * kMaxDiagCtrl * D);
  std::vector<double2> hv((size_t)(K + 1) * W * D, double2{0.0, 0.0});
  std::vector<double2> hk((size_t)std::max(K, 1) * kMaxDiagCtrl * D, double2{0.0, 0.0});
  for (size_t i = 0; i < D; ++i) {
    const std::vector<int64_t>& v = rc[i];
    for (int e = 0; e < W; ++e) hc[(size_t)e * D + i] = (int32_t)(e < (int)v.size() ? v[e] : (int64_t)i);
    for (int o = 0; o <= K; ++o)
      for (auto& en : ops[o][i]) {
        // slot of the column; a complex main diagonal skips the stand-in slot 0
        int e = (en.col == (int64_t)i && !diag_complex) ? 0 : 1;
        while (v[e] != en.col) ++e;
        hv[((size_t)o * W + e) * D + i] = double2{en.re, en.im};
      }
    for (int k = 0; k < K; ++k) {
      int qq = 0;
      for (auto& en : ops[k + 1][i]) {
        hck[((size_t)k * kMaxDiagCtrl + qq) * D + i] = (int32_t)en.col;
        hk[((size_t)k * kMaxDiagCtrl + qq) * D + i] = double2{en.re, en.im};
        ++qq;
      }
      for (; qq < kMaxDiagCtrl; ++qq) hck[((size_t)k * kMaxDiagCtrl + qq) * D + i] = (int32_t)i;
    }
  }
  HG_HIP(hipMalloc(&d.vals, hv.size() * sizeof(double2)));
  HG_HIP(hipMemcpy(d.vals, hv.data(), hv.size() * sizeof(double2), hipMemcpyHostToDevice));
  HG_HIP(hipMalloc(&d.valk, hk.size() * sizeof(double2)));
  HG_HIP(hipMemcpy(d.valk, hk.data(), hk.size() * sizeof(double2), hipMemcpyHostToDevice));
  HG_HIP(hipMalloc(&d.cols, hc.size() * sizeof(int32_t)));
  HG_HIP(hipMemcpy(d.cols, hc.data(), hc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HG_HIP(hipMalloc(&d.colk, hck.size() * sizeof(int32_t)));
  HG_HIP(hipMemcpy(d.colk, hck.data(), hck.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (omega_diag) {
    HG_HIP(hipMalloc(&d.omega, dim * sizeof(double)));
    HG_HIP(hipMemcpy(d.omega, omega_diag, dim * sizeof(double), hipMemcpyHostToDevice));
  }
  SweepShape sh{};
  std::string w64, w128;
  const bool one64 = dim <= (int64_t)kMaxThreads * kMaxRows &&
                     sweep_supported(d, (int)dim, K, false, ctx->lds_per_block, &sh, &w64);
  const bool one128 = dim <= (int64_t)kMaxThreads * kMaxRows &&
                      sweep_supported(d, (int)dim, K, true, ctx->lds_per_block, &sh, &w128);
  if (!one64 && !one128)
    return fail(HG_ERR_UNSUPPORTED, "row-indexed storage: " + w64);
  *out = p.release();
  return HG_OK;
}

static hg_status problem_create_impl(hg_ctx* ctx, int64_t dim, int32_t n_ctrl, const hg_csr* H0,
                            const hg_csr* Hk, const double* omega_diag, bool dense,
                            hg_problem** out) {
  if (!ctx || !out || !H0) return fail(HG_ERR_INVALID_ARG, "NULL argument");
  const int64_t dmax = dense ? (int64_t)kDenseMaxDim : (int64_t)kMaxDimSplit;
  if (dim < 1 || dim > dmax)
    return fail(dim < 1 ? HG_ERR_INVALID_ARG : HG_ERR_UNSUPPORTED,
                "dim must be in [1, " + std::to_string(dmax) + "]");
  if (n_ctrl < 0 || n_ctrl > kMaxCtrl)
    return fail(n_ctrl < 0 ? HG_ERR_INVALID_ARG : HG_ERR_UNSUPPORTED, "n_ctrl out of range");
  if (n_ctrl > 0 && !Hk) return fail(HG_ERR_INVALID_ARG, "Hk is NULL");
  HG_HIP(hipSetDevice(ctx->device));

  const int K = n_ctrl;
  std::vector<std::vector<std::vector<Entry>>> ops(K + 1);
  hg_status st = read_csr(H0, dim, "H0", &ops[0]);
  if (st != HG_OK) return st;
  if ((st = check_hermitian(ops[0], "H0")) != HG_OK) return st;
  for (int k = 0; k < K; ++k) {
    const std::string nm = "H" + std::to_string(k + 1);
    if ((st = read_csr(&Hk[k], dim, nm.c_str(), &ops[k + 1])) != HG_OK) return st;
    if ((st = check_hermitian(ops[k + 1], nm.c_str())) != HG_OK) return st;
  }
  if (omega_diag)
    for (int64_t i = 0; i < dim; ++i)
      if (!std::isfinite(omega_diag[i])) return fail(HG_ERR_NONFINITE, "omega: non-finite value");

  // union diagonals, per-control diagonals, sigma' and structural counts
  std::set<int64_t> uoff;
  std::vector<std::set<int64_t>> koff(K);
  int64_t sigma = 0, nnz = 0;
  std::vector<int64_t> nnz_ctrl(K, 0);
  std::set<int64_t> complex_off;  // offsets with a non-zero imaginary part in some operator
  for (int64_t i = 0; i < dim; ++i) {
    std::set<int64_t> cols;
    for (int o = 0; o <= K; ++o)
      for (auto& e : ops[o][i]) {
        cols.insert(e.col);
        uoff.insert(e.col - i);
        if (e.im != 0.0) complex_off.insert(e.col - i);
        if (o > 0) {
          koff[o - 1].insert(e.col - i);
          nnz_ctrl[o - 1]++;
        }
      }
    sigma = std::max<int64_t>(sigma, (int64_t)cols.size());
    nnz += (int64_t)cols.size();
  }
  if (uoff.empty()) uoff.insert(0);
  if (dense) {
    // dense storage: H[o][i][j] row-major, padded to dp = dim rounded up to 64
    auto p = std::make_unique<hg_problem>();
    p->ctx = ctx;
    p->dim = dim;
    p->n_ctrl = K;
    p->sigma = (int32_t)std::max<int64_t>(sigma, 1);
    p->nnz = nnz;
    p->nnz_ctrl = nnz_ctrl;
    p->dense = true;
    p->dp = (dim + 63) / 64 * 64;
    const size_t dp = (size_t)p->dp, plane = dp * dp;
    std::vector<double2> hd((size_t)(K + 1) * plane, double2{0.0, 0.0});
    for (int o = 0; o <= K; ++o)
      for (int64_t i = 0; i < dim; ++i)
        for (auto& en : ops[o][i]) hd[(size_t)o * plane + (size_t)i * dp + en.col] = double2{en.re, en.im};
    if (hipMalloc(&p->dops.H, hd.size() * sizeof(double2)) != hipSuccess)
      return fail(HG_ERR_OUT_OF_MEMORY, "dense operators: " + std::to_string(hd.size() * 16) + " bytes");
    HG_HIP(hipMemcpy(p->dops.H, hd.data(), hd.size() * sizeof(double2), hipMemcpyHostToDevice));
    if (omega_diag) {
      HG_HIP(hipMalloc(&p->ops.omega, dim * sizeof(double)));
      HG_HIP(hipMemcpy(p->ops.omega, omega_diag, dim * sizeof(double), hipMemcpyHostToDevice));
      p->dops.omega = p->ops.omega;
    }
    *out = p.release();
    return HG_OK;
  }
  // Union order: the main diagonal first, then the other diagonals on which
  // every operator is real (B = -i dt/s H is purely imaginary there, so its
  // products take half the multiply-adds), then the rest.  A main diagonal
  // that is absent, or complex somewhere, keeps slot 0 as an all-zero
  // diagonal and goes to a slot of its own at the end, so slot 0 is always
  // purely imaginary.
  const bool diag_slot = !uoff.count(0) || complex_off.count(0);
  std::vector<int64_t> order{0};
  for (int64_t o : uoff)
    if (o != 0 && !complex_off.count(o)) order.push_back(o);
  const int npure = (int)order.size();
  for (int64_t o : uoff)
    if (o != 0 && complex_off.count(o)) order.push_back(o);
  if (diag_slot && uoff.count(0)) order.push_back(0);
  bool wide_ctrl = false;
  for (int k = 0; k < K; ++k) wide_ctrl = wide_ctrl || (int)koff[k].size() > kMaxDiagCtrl;
  if ((int)order.size() > kMaxDiagKernels || wide_ctrl)
    return create_ell(ctx, dim, K, ops, omega_diag, complex_off.count(0) > 0, sigma, nnz, nnz_ctrl,
                      out);

  auto p = std::make_unique<hg_problem>();
  p->ctx = ctx;
  p->dim = dim;
  p->n_ctrl = K;
  p->sigma = (int32_t)std::max<int64_t>(sigma, 1);
  p->nnz = nnz;
  p->nnz_ctrl = nnz_ctrl;
  DevOps& d = p->ops;
  d.W = (int)order.size();
  d.npure = npure;
  classify_controls(ops, dim, K, &d);
  std::map<int64_t, int> slot;
  for (int e = 0; e < d.W; ++e) {
    d.off[e] = (int)order[e];
    slot[order[e]] = e;  // a complex main diagonal maps to its own (last) slot
    d.halo = std::max<int>(d.halo, (int)std::llabs(order[e]));
  }
  for (int k = 0; k < K; ++k) {
    d.WK[k] = (int)koff[k].size();
    int q = 0;
    for (int64_t o : koff[k]) d.offk[k][q++] = (int)o;
  }
  std::vector<double2> hv((size_t)(K + 1) * d.W * dim, double2{0.0, 0.0});
  std::vector<double2> hk((size_t)std::max(K, 1) * kMaxDiagCtrl * dim, double2{0.0, 0.0});
  for (int o = 0; o <= K; ++o)
    for (int64_t i = 0; i < dim; ++i)
      for (auto& en : ops[o][i]) {
        const int64_t off = en.col - i;
        hv[((size_t)o * d.W + slot[off]) * dim + i] = double2{en.re, en.im};
        if (o > 0) {
          int q = 0;
          while (d.offk[o - 1][q] != off) ++q;
          hk[((size_t)(o - 1) * kMaxDiagCtrl + q) * dim + i] = double2{en.re, en.im};
        }
      }
  HG_HIP(hipMalloc(&d.vals, hv.size() * sizeof(double2)));
  HG_HIP(hipMemcpy(d.vals, hv.data(), hv.size() * sizeof(double2), hipMemcpyHostToDevice));
  HG_HIP(hipMalloc(&d.valk, hk.size() * sizeof(double2)));
  HG_HIP(hipMemcpy(d.valk, hk.data(), hk.size() * sizeof(double2), hipMemcpyHostToDevice));
  if (omega_diag) {
    HG_HIP(hipMalloc(&d.omega, dim * sizeof(double)));
    HG_HIP(hipMemcpy(d.omega, omega_diag, dim * sizeof(double), hipMemcpyHostToDevice));
  }
  // Rows beyond one workgroup (in either precision): split the columns.
  {
    SweepShape sh{};
    std::string w64, w128;
    const bool one64 = dim <= (int64_t)kMaxThreads * kMaxRows &&
                       sweep_supported(d, (int)dim, K, false, ctx->lds_per_block, &sh, &w64);
    const bool one128 = dim <= (int64_t)kMaxThreads * kMaxRows &&
                        sweep_supported(d, (int)dim, K, true, ctx->lds_per_block, &sh, &w128);
    if (!one64 || !one128) {
      Split& sp = p->split;
      std::string why;
      if (!plan_split(ops, dim, d, K, ctx->lds_per_block, ctx->num_cu, &sp, &why)) {
        sp = Split{};
        if (!one64 && !one128)
          return fail(HG_ERR_UNSUPPORTED, "dimension " + std::to_string(dim) +
                                              " does not fit one workgroup and " + why);
      } else {
        const size_t dl = (size_t)sp.d_loc, P = (size_t)sp.P, W = (size_t)d.W;
        sp.vals_stride = (size_t)(K + 1) * W * dl;
        sp.valk_stride = (size_t)std::max(K, 1) * kMaxDiagCtrl * dl;
        sp.omega_stride = dl;
        std::vector<double2> lv(P * sp.vals_stride, double2{0.0, 0.0});
        std::vector<double2> lk(P * sp.valk_stride, double2{0.0, 0.0});
        std::vector<double> lo(P * dl, 0.0);
        for (int q = 0; q < sp.P; ++q)
          for (int t = 0; t < sp.T; ++t)
            for (int k = 0; k < sp.w[q]; ++k) {
              const size_t l = (size_t)t * sp.seg + sp.h + k;
              const size_t gi = (size_t)t * sp.L + sp.c0[q] + k;
              for (int o = 0; o <= K; ++o)
                for (size_t e2 = 0; e2 < W; ++e2)
                  lv[q * sp.vals_stride + ((size_t)o * W + e2) * dl + l] = hv[((size_t)o * W + e2) * dim + gi];
              for (int k2 = 0; k2 < K; ++k2)
                for (int qq = 0; qq < kMaxDiagCtrl; ++qq)
                  lk[q * sp.valk_stride + ((size_t)k2 * kMaxDiagCtrl + qq) * dl + l] =
                      hk[((size_t)k2 * kMaxDiagCtrl + qq) * dim + gi];
              if (omega_diag) lo[q * dl + l] = omega_diag[gi];
            }
        HG_HIP(hipMalloc(&sp.ops.vals, lv.size() * sizeof(double2)));
        HG_HIP(hipMemcpy(sp.ops.vals, lv.data(), lv.size() * sizeof(double2), hipMemcpyHostToDevice));
        HG_HIP(hipMalloc(&sp.ops.valk, lk.size() * sizeof(double2)));
        HG_HIP(hipMemcpy(sp.ops.valk, lk.data(), lk.size() * sizeof(double2), hipMemcpyHostToDevice));
        if (omega_diag) {
          HG_HIP(hipMalloc(&sp.ops.omega, lo.size() * sizeof(double)));
          HG_HIP(hipMemcpy(sp.ops.omega, lo.data(), lo.size() * sizeof(double), hipMemcpyHostToDevice));
        }
      }
    }
  }
  *out = p.release();
  return HG_OK;
}

hg_status hg_problem_destroy(hg_problem* p) {
  delete p;
  return HG_OK;
}

hg_status hg_problem_info(const hg_problem* p, int64_t* dim, int32_t* n_ctrl, int32_t* ell_width,
                          int32_t* sigma, int64_t* nnz) {
  if (!p) return fail(HG_ERR_INVALID_ARG, "problem is NULL");
  if (dim) *dim = p->dim;
  if (n_ctrl) *n_ctrl = p->n_ctrl;
  if (ell_width) *ell_width = p->dense ? 0 : p->ops.W;
  if (sigma) *sigma = p->sigma;
  if (nnz) *nnz = p->nnz;
  return HG_OK;
}

double hg_error_bound(double theta, int32_t m, int32_t s, int32_t sigma, double u) {
  if (m < 1 || s < 1 || sigma < 1 || !(theta >= 0.0)) return std::nan("");
  return error_bound(theta, m, s, sigma, u);
}

static hg_status plan_impl(const double* theta, int64_t n, int32_t sigma, double tau, double u,
                           int32_t* m_out, int32_t* s_out, bool table = true,
                           int rule = HG_PLAN_SMALLEST_S) {
  if (n < 0 || (n > 0 && (!theta || !m_out || !s_out)) || sigma < 1 || !(tau > 0.0) ||
      !(u > 0.0 && u < 0.25))
    return fail(HG_ERR_INVALID_ARG, "hg_plan: bad argument");
  if (rule != HG_PLAN_SMALLEST_S && rule != HG_PLAN_MIN_MU)
    return fail(HG_ERR_INVALID_ARG, "hg_plan: unknown rule");
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(theta[i])) return fail(HG_ERR_NONFINITE, "norm " + std::to_string(i) + " is not finite");
    if (theta[i] < 0.0) return fail(HG_ERR_INVALID_ARG, "negative norm");
  }
  int64_t bad = -1;
  const int rc = plan_steps(theta, n, sigma, tau, u, m_out, s_out, &bad, table, rule);
  if (rc == 2)
    return fail(HG_ERR_UNSUPPORTED, "step " + std::to_string(bad) + " (norm " +
                                        std::to_string(theta[bad]) + ") would need s > " +
                                        std::to_string(kSMax) + "; shorten dt");
  if (rc != 0) {
    char buf[256];
    std::snprintf(buf, sizeof(buf),
                  "no (m<=%d, s) meets E_A <= %g at step %lld (norm %.6g); the rounding floor of "
                  "the bound exceeds the tolerance",
                  kMMax, tau, (long long)bad, theta[bad]);
    return fail(HG_ERR_TOLERANCE_UNREACHABLE, buf);
  }
  return HG_OK;
}

hg_status hg_step_norms(hg_problem* p, const double* u, int32_t n_batch, int32_t n_steps,
                        double dt, double* theta_out, void* stream) {
  if (!p || !u || !theta_out || n_batch < 1 || n_steps < 1)
    return fail(HG_ERR_INVALID_ARG, "hg_step_norms: bad argument");
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(HG_ERR_INVALID_ARG, "dt must be finite and > 0");
  HG_HIP(hipSetDevice(p->ctx->device));
  if (p->dense)
    HG_HIP(launch_dense_norms(p->dops, (int)p->dim, (int)p->dp, p->n_ctrl, u, n_batch, n_steps, dt,
                              theta_out, (hipStream_t)stream));
  else
    HG_HIP(launch_step_norms(p->ops, (int)p->dim, p->n_ctrl, u, n_batch, n_steps, dt, theta_out,
                             (hipStream_t)stream));
  return HG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// HG_METHOD_AUTO: diagonalise when mean(mu) * S >= c (d + S).  The constants
// come from the measured crossover on the three-transmon gate (d = S = 216 and
// 512): the Jacobi eigensolver runs in FP64 for both precisions while the
// complex64 Taylor products run twice as fast as the complex128 ones.
constexpr double kAutoDiagC128 = 40.0;
constexpr double kAutoDiagC64 = 200.0;

struct Workspace {
  size_t theta, pnorm, sched, psiN, cold, ckpt, segbuf, ovl, ovt, gt, pen, gradp, drift, res;
  size_t mat, emat, blocks;  // dense path
  size_t psi0_loc, tgt_loc, xbuf, xnrm, xflag, xerr;  // split columns
  size_t diag;                                         // diagonalisation method
  size_t total;
};

// Workgroups per state column for this problem and precision: 1 when one
// workgroup holds a column, else the problem's split (0 if neither works).
static int parts_for(const hg_problem* p, bool c128) {
  if (p->dense) return 1;
  SweepShape sh{};
  std::string why;
  if (p->dim <= (int64_t)kMaxThreads * kMaxRows &&
      sweep_supported(p->ops, (int)p->dim, p->n_ctrl, c128, p->ctx->lds_per_block, &sh, &why))
    return 1;
  return p->split.P > 1 ? p->split.P : 0;
}

static DenseShape dense_shape(const hg_problem* p, int B, int N, int S, bool c128) {
  DenseShape sh{};
  sh.d = (int)p->dim;
  sh.dp = (int)p->dp;
  sh.K = p->n_ctrl;
  sh.N = N;
  sh.S = S;
  sh.Sp = (S + 63) / 64 * 64;
  sh.B = B;
  sh.c128 = c128;
  sh.num_cu = p->ctx->num_cu;
  return sh;
}

static Workspace layout(const hg_problem* p, int B, int N, int S_true, bool c128, int ckpt_every,
                        bool integrated, int Q = 1, int method = HG_METHOD_TAYLOR) {
  const size_t cs = c128 ? 16 : 8;
  const int parts = std::max(parts_for(p, c128), 1);
  // a split column is P local columns of d_loc rows each
  const size_t d = parts > 1 ? (size_t)p->split.d_loc : (size_t)p->dim, K = (size_t)p->n_ctrl;
  const int S = S_true * parts;
  Workspace w{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  w.theta = take((size_t)B * N * 8);
  w.pnorm = take((size_t)B * S_true * 8);
  w.sched = take((size_t)2 * B * N * 4);
  const bool dn = p->dense;
  w.psiN = take(dn ? 0 : (size_t)B * S * d * cs);
  w.cold = take(dn ? 0 : (size_t)B * S * Q * 3 * d * 16);  // FP64 carried vectors
  const size_t C = ckpt_every > 0 ? (size_t)std::min(ckpt_every, N) : 0;
  const size_t nseg = ckpt_every > 0 ? ((size_t)N + ckpt_every - 1) / ckpt_every : 0;
  w.ckpt = take(dn ? 0 : (size_t)B * S * nseg * d * cs);
  w.segbuf = take(dn ? 0 : (size_t)B * S * Q * C * d * cs);
  w.ovl = take((size_t)B * S * 16);
  w.ovt = take(integrated ? (size_t)B * S * N * 16 : 0);
  w.gt = take(integrated ? (size_t)B * N * 16 : 0);
  w.pen = take((size_t)B * S * 8);
  w.gradp = take(dn ? 0 : (size_t)B * S * std::max<size_t>(K, 1) * N * 8);
  w.drift = take((size_t)B * S * 8);
  w.res = take((size_t)B * 8 * 8);
  if (parts > 1) {
    const Split& sp = p->split;
    w.psi0_loc = take((size_t)B * S * d * 16);
    w.tgt_loc = take((size_t)B * S * d * 16);
    w.xbuf = take((size_t)B * S * 4 * sp.T * std::max(sp.h, 1) * 64);
    w.xnrm = take((size_t)B * S * kMaxParts * 8);
    w.xflag = take((size_t)B * S * 4);
    w.xerr = take(4);
  }
  if (dn) {
    const DenseShape sh = dense_shape(p, B, N, S, c128);
    if (method != HG_METHOD_DIAG) {  // Taylor products on the matrix cores (AUTO may take either)
      const size_t rs = cs / 2, Mp = 2 * (size_t)sh.dp;
      w.mat = take((size_t)B * Mp * Mp * rs);
      w.emat = take((size_t)B * K * Mp * Mp * rs);
      w.blocks = take(dense_block_elems(sh) * rs);
      // checkpoint variant: whole state groups (padded columns, embedded rows)
      const size_t grp = (size_t)sh.Sp * Mp * rs;
      w.ckpt = take((size_t)B * nseg * grp);
      w.segbuf = take((size_t)B * C * grp);
    }
    if (method != HG_METHOD_TAYLOR) w.diag = take(diag_work_bytes(sh));
  }
  w.total = o;
  return w;
}

static hg_status check_desc(const hg_problem* p, const hg_eval_desc* d) {
  if (!p || !d) return fail(HG_ERR_INVALID_ARG, "NULL problem or desc");
  if (d->n_steps < 1) return fail(HG_ERR_INVALID_ARG, "n_steps must be >= 1");
  if (d->n_batch < 1) return fail(HG_ERR_INVALID_ARG, "n_batch must be >= 1");
  if (d->n_states < 1) return fail(HG_ERR_INVALID_ARG, "n_states must be >= 1");
  if (!std::isfinite(d->dt) || !(d->dt > 0.0)) return fail(HG_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (!std::isfinite(d->w_fid) || !std::isfinite(d->w_pen) || !std::isfinite(d->w_int))
    return fail(HG_ERR_NONFINITE, "weights");
  if (!(d->tau > 0.0) || !std::isfinite(d->tau)) return fail(HG_ERR_INVALID_ARG, "tau must be > 0");
  if (d->dtype != HG_C64 && d->dtype != HG_C128) return fail(HG_ERR_INVALID_ARG, "dtype");
  if (d->mode != HG_MODE_RECONSTRUCT && d->mode != HG_MODE_CHECKPOINT)
    return fail(HG_ERR_INVALID_ARG, "mode");
  if (d->mode == HG_MODE_CHECKPOINT && d->ckpt_every < 1)
    return fail(HG_ERR_INVALID_ARG, "checkpoint mode needs ckpt_every >= 1");
  if (d->renorm_every < 0) return fail(HG_ERR_INVALID_ARG, "renorm_every must be >= 0");
  if (d->rule != HG_PLAN_SMALLEST_S && d->rule != HG_PLAN_MIN_MU)
    return fail(HG_ERR_INVALID_ARG, "unknown planner rule");
  if (d->method != HG_METHOD_TAYLOR && d->method != HG_METHOD_DIAG && d->method != HG_METHOD_AUTO)
    return fail(HG_ERR_INVALID_ARG, "unknown method");
  if (d->method == HG_METHOD_DIAG && !p->dense)
    return fail(HG_ERR_UNSUPPORTED, "the diagonalisation method needs dense operator storage "
                                    "(hg_problem_create_dense)");
  if ((p->n_ctrl > 0 && !d->u) || !d->psi0 || !d->targets)
    return fail(HG_ERR_INVALID_ARG, "NULL device array");
  if (p->dense && d->mode == HG_MODE_CHECKPOINT && d->method == HG_METHOD_DIAG)
    return fail(HG_ERR_UNSUPPORTED, "the diagonalisation method rebuilds states exactly; the "
                                    "checkpoint mode is built for the Taylor method");
  return HG_OK;
}

static hg_status shape_for(const hg_problem* p, const hg_eval_desc* d, SweepShape* sh);

hg_status hg_eval_footprint(const hg_problem* p, const hg_eval_desc* d, size_t* bytes) {
  hg_status st = check_desc(p, d);
  if (st != HG_OK) return st;
  if (!bytes) return fail(HG_ERR_INVALID_ARG, "bytes is NULL");
  SweepShape sh{};
  sh.spread = 1;
  if (shape_for(p, d, &sh) != HG_OK) sh.spread = 1;  // the evaluation itself reports it
  *bytes = layout(p, d->n_batch, d->n_steps, d->n_states, d->dtype == HG_C128,
                  d->mode == HG_MODE_CHECKPOINT ? d->ckpt_every : 0,
                  d->w_int != 0.0, sh.spread, p->dense ? d->method : HG_METHOD_TAYLOR).total;
  return HG_OK;
}

// Bytes of host staging one evaluation needs: norms, state norms, schedule,
// result scalars and drifts.
static size_t host_stage_bytes(int B, int N, int S, int parts) {
  return (size_t)B * N * 8 + (size_t)B * S * 8 + (size_t)2 * B * N * 4 + (size_t)B * 8 * 8 +
         (size_t)B * S * parts * 8 + 8 + (size_t)B * 8;
}

// The evaluation proper, on a workspace `ws` laid out by layout() and a host
// staging area `hbuf` of host_stage_bytes() (pinned or pageable).  `table`
// lets the planner build and cache its threshold table; without it the planner
// uses a cached table if there is one, else the direct search (same decisions).
static hg_status eval_core(hg_problem* p, const hg_eval_desc* d, hg_result* results, double* grad,
                           hipStream_t hs, const SweepShape& sh0, const Workspace& w, char* ws,
                           char* hbuf, bool table) {
  const int B = d->n_batch, N = d->n_steps, S = d->n_states, K = p->n_ctrl;
  const bool c128 = d->dtype == HG_C128;
  hg_status st = HG_OK;
  SweepShape sh = sh0;
  const int ck = d->mode == HG_MODE_CHECKPOINT ? std::min(d->ckpt_every, N) : 0;
  struct Drain {  // on an early return, copies into the staging area may still be queued
    hipStream_t s;
    bool armed = true;
    ~Drain() {
      if (armed) (void)hipStreamSynchronize(s);
    }
  } drain{hs};
  double* h_theta = (double*)hbuf;
  double* h_pnorm = h_theta + (size_t)B * N;
  int32_t* h_sched = (int32_t*)(h_pnorm + (size_t)B * S);
  double* h_res = (double*)(h_sched + (size_t)2 * B * N);
  double* h_drift = h_res + (size_t)B * 8;
  const int parts = std::max(sh.parts, 1);
  uint32_t* h_xerr = (uint32_t*)(h_drift + (size_t)B * S * parts);
  int* h_done = (int*)(h_xerr + 2);

  double* d_theta = (double*)(ws + w.theta);
  double* d_pnorm = (double*)(ws + w.pnorm);
  int32_t* d_sched = (int32_t*)(ws + w.sched);
  const double* u_dev = d->u;
  if (K == 0) u_dev = d_theta;  // never read (no controls); any valid pointer

  // 1-norms of every step (App. C) and state norms, then the host planner
  if (p->dense)
    HG_HIP(launch_dense_norms(p->dops, (int)p->dim, (int)p->dp, K, u_dev, B, N, d->dt, d_theta, hs));
  else
    HG_HIP(launch_step_norms(p->ops, (int)p->dim, K, u_dev, B, N, d->dt, d_theta, hs));
  HG_HIP(launch_state_norms(d->psi0, (int)p->dim, S, B, d_pnorm, hs));
  HG_HIP(hipMemcpyAsync(h_theta, d_theta, (size_t)B * N * 8, hipMemcpyDeviceToHost, hs));
  HG_HIP(hipMemcpyAsync(h_pnorm, d_pnorm, (size_t)B * S * 8, hipMemcpyDeviceToHost, hs));
  HG_HIP(hipStreamSynchronize(hs));
  for (int64_t i = 0; i < (int64_t)B * S; ++i)
    if (!std::isfinite(h_pnorm[i]) || std::fabs(h_pnorm[i] - 1.0) > 1e-8)
      return fail(std::isfinite(h_pnorm[i]) ? HG_ERR_INVALID_ARG : HG_ERR_NONFINITE,
                  "initial state " + std::to_string(i) + " has norm " + std::to_string(h_pnorm[i]) +
                      " (must be 1 to 1e-8)");
  for (int64_t i = 0; i < (int64_t)B * N; ++i)
    if (!std::isfinite(h_theta[i]))
      return fail(HG_ERR_NONFINITE, "amplitudes of step " + std::to_string(i % N) + " are not finite");
  int32_t* h_m = h_sched;
  int32_t* h_s = h_sched + (size_t)B * N;
  const bool diag_only = p->dense && d->method == HG_METHOD_DIAG;
  if (diag_only) {
    // no Taylor products: no schedule (sum_mu and the bound are reported as 0)
    for (int64_t i = 0; i < (int64_t)B * N; ++i) h_m[i] = h_s[i] = 0;
  } else if (d->schedule) {
    for (int64_t i = 0; i < (int64_t)B * N; ++i) {
      h_m[i] = d->schedule[i];
      h_s[i] = d->schedule[(size_t)B * N + i];
      if (h_m[i] < 1 || h_m[i] > kMMax || h_s[i] < 1 || h_s[i] > kSMax)
        return fail(HG_ERR_INVALID_ARG, "frozen schedule entry " + std::to_string(i) + " out of range");
    }
  } else {
    // FP64 arithmetic bound (u = 2^-53) for both precisions: the schedule is
    // chosen by the paper's rule for double arithmetic; complex64 then differs
    // from complex128 only in the arithmetic of the products.
    st = plan_impl(h_theta, (int64_t)B * N, p->sigma, d->tau, std::ldexp(1.0, -53), h_m, h_s,
                   table, d->rule);
    if (st != HG_OK) return st;
  }
  HG_HIP(hipMemcpyAsync(d_sched, h_sched, (size_t)2 * B * N * 4, hipMemcpyHostToDevice, hs));
  bool use_diag = diag_only;
  if (p->dense && d->method == HG_METHOD_AUTO) {
    // Sec. V: the Taylor products cost ~ mu d^2 S per step, diagonalisation
    // ~ d^3 + d^2 S; take the diagonalisation when mean mu * S >= c (d + S)
    double mu = 0.0;
    for (int64_t i = 0; i < (int64_t)B * N; ++i) mu += (double)h_m[i] * h_s[i];
    mu /= (double)B * N;
    use_diag = ck == 0 && mu * S >= (c128 ? kAutoDiagC128 : kAutoDiagC64) * ((double)p->dim + S);
  }

  SweepBuffers bf{};
  bf.u = u_dev;
  bf.m_sched = d_sched;
  bf.s_sched = d_sched + (size_t)B * N;
  bf.psi0 = d->psi0;
  bf.targets = d->targets;
  bf.psiN = ws + w.psiN;
  bf.cold = ws + w.cold;
  bf.ckpt = ck > 0 ? ws + w.ckpt : nullptr;
  bf.segbuf = ck > 0 ? ws + w.segbuf : nullptr;
  bf.ovl = (double*)(ws + w.ovl);
  bf.ovt = d->w_int != 0.0 ? (double*)(ws + w.ovt) : nullptr;
  bf.gt = d->w_int != 0.0 ? (double*)(ws + w.gt) : nullptr;
  bf.pen = (double*)(ws + w.pen);
  bf.gradp = (double*)(ws + w.gradp);
  bf.drift = (double*)(ws + w.drift);
  bf.res = (double*)(ws + w.res);
  bf.grad = grad;
  bf.ev[0] = bf.ev[1] = bf.ev[2] = nullptr;
  struct Events {
    hipEvent_t* e;
    ~Events() {
      for (int i = 0; i < 3; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } evguard{bf.ev};
  if (d->flags & HG_FLAG_TIMING)
    for (int i = 0; i < 3; ++i) HG_HIP(hipEventCreate(&bf.ev[i]));
  SweepParams sp{d->dt, d->w_fid, d->w_pen, d->w_int, d->renorm_every, ck};
  if (p->dense && use_diag) {
    DiagBuffers db{};
    db.u = u_dev;
    db.psi0 = d->psi0;
    db.targets = d->targets;
    db.work = ws + w.diag;
    db.h_done = h_done;
    db.pen = bf.pen;
    db.ovl = bf.ovl;
    db.ovt = bf.ovt;
    db.gt = bf.gt;
    db.drift = bf.drift;
    db.res = bf.res;
    db.grad = grad;
    for (int i = 0; i < 3; ++i) db.ev[i] = bf.ev[i];
    HG_HIP(launch_diag_sweep(p->ctx->device, p->dops, dense_shape(p, B, N, S, c128), db, sp, hs));
  } else if (p->dense) {
    DenseBuffers db{};
    db.u = u_dev;
    db.m_sched = bf.m_sched;
    db.s_sched = bf.s_sched;
    db.psi0 = d->psi0;
    db.targets = d->targets;
    db.blocks = ws + w.blocks;
    db.mat = ws + w.mat;
    db.emat = ws + w.emat;
    db.ckpt = ck > 0 ? ws + w.ckpt : nullptr;
    db.segbuf = ck > 0 ? ws + w.segbuf : nullptr;
    db.pen = bf.pen;
    db.ovl = bf.ovl;
    db.ovt = bf.ovt;
    db.gt = bf.gt;
    db.drift = bf.drift;
    db.res = bf.res;
    db.grad = grad;
    for (int i = 0; i < 3; ++i) db.ev[i] = bf.ev[i];
    HG_HIP(launch_dense_sweep(p->dops, dense_shape(p, B, N, S, c128), db, sp, h_m, h_s, hs));
  } else if (parts > 1) {
    SplitBuffers x{};
    x.psi0_loc = (double2*)(ws + w.psi0_loc);
    x.tgt_loc = (double2*)(ws + w.tgt_loc);
    x.xbuf = (unsigned char*)(ws + w.xbuf);
    x.xnrm = (double*)(ws + w.xnrm);
    x.xflag = (uint32_t*)(ws + w.xflag);
    x.xerr = (uint32_t*)(ws + w.xerr);
    HG_HIP(launch_split_sweep(p->split, sh, bf, x, sp, S, hs));
    HG_HIP(hipMemcpyAsync(h_xerr, x.xerr, 4, hipMemcpyDeviceToHost, hs));
  } else {
    HG_HIP(launch_sweep(p->ops, sh, bf, sp, hs));
  }
  HG_HIP(hipMemcpyAsync(h_res, bf.res, (size_t)B * 8 * 8, hipMemcpyDeviceToHost, hs));
  HG_HIP(hipMemcpyAsync(h_drift, bf.drift, (size_t)B * S * parts * 8, hipMemcpyDeviceToHost, hs));
  HG_HIP(hipStreamSynchronize(hs));
  drain.armed = false;
  if (parts > 1 && *h_xerr != 0)
    return fail(HG_ERR_DEVICE, "split-column sweep: a workgroup waited too long for the halo rows "
                               "of its neighbour (are other kernels holding the compute units?)");
  float ms_f = 0.f, ms_b = 0.f;
  if (d->flags & HG_FLAG_TIMING) {
    HG_HIP(hipEventElapsedTime(&ms_f, bf.ev[0], bf.ev[1]));
    HG_HIP(hipEventElapsedTime(&ms_b, bf.ev[1], bf.ev[2]));
  }

  for (int b = 0; b < B; ++b) {
    hg_result& r = results[b];
    r.cost = h_res[b * 8 + 0];
    r.infidelity = h_res[b * 8 + 1];
    r.penalty = h_res[b * 8 + 2];
    r.integrated_infidelity = h_res[b * 8 + 5];
    r.overlap_re = h_res[b * 8 + 3];
    r.overlap_im = h_res[b * 8 + 4];
    int64_t mu = 0;
    double mt = 0.0, mb = 0.0, dr = 0.0;
    // E_A(m, s, theta) grows with theta for fixed (m, s), so the largest bound
    // is found by evaluating it once per (m, s) pair at the largest norm
    // planned with that pair: a handful of evaluations instead of N (a fixed
    // table, no allocation; pairs beyond it are evaluated step by step)
    struct PairTop {
      int32_t m, s;
      double theta;
    };
    PairTop top[32];
    int ntop = 0;
    const double u53 = std::ldexp(1.0, -53);
    for (int n = 0; n < N; ++n) {
      const size_t i = (size_t)b * N + n;
      if (!use_diag) mu += (int64_t)h_m[i] * h_s[i];
      mt = std::max(mt, h_theta[i]);
      if (!d->schedule && !use_diag) {
        int q = 0;
        while (q < ntop && (top[q].m != h_m[i] || top[q].s != h_s[i])) ++q;
        if (q < ntop)
          top[q].theta = std::max(top[q].theta, h_theta[i]);
        else if (ntop < 32)
          top[ntop++] = PairTop{h_m[i], h_s[i], h_theta[i]};
        else
          mb = std::max(mb, error_bound(h_theta[i], h_m[i], h_s[i], p->sigma, u53));
      }
    }
    for (int q = 0; q < ntop; ++q)
      mb = std::max(mb, error_bound(top[q].theta, top[q].m, top[q].s, p->sigma, u53));
    for (int h = 0; h < S; ++h) {
      // a split column's parts hold disjoint rows: combine their partial drifts
      double d2 = 0.0;
      for (int q = 0; q < parts; ++q) {
        const double x = h_drift[((size_t)b * S + h) * parts + q];
        d2 += x * x;
      }
      dr = std::max(dr, parts > 1 ? std::sqrt(d2) : h_drift[(size_t)b * S + h]);
    }
    r.sum_mu = mu;
    r.max_theta = mt;
    r.max_bound = mb;
    r.drift = dr;
    r.ms_forward = ms_f;
    r.ms_backward = ms_b;
  }
  return HG_OK;
}


// With HG_FLAG_SPREAD: the control group size and the number of backward
// workgroups per column that minimise the estimated backward time when the
// batch's B*S columns leave compute units idle.  Per Taylor term, phase 1
// costs 2 products with the union operator; a phase-2 pass with g controls
// costs 1 + g of them plus g control products (relative cost e).  Larger g
// wins ties (less repeated work).
static void choose_spread(const hg_problem* p, const hg_eval_desc* d, SweepShape* sh) {
  sh->spread = 1;
  const int K = p->n_ctrl;
  if (!(d->flags & HG_FLAG_SPREAD) || p->dense || sh->parts > 1 || K < 2) return;
  const int budget = p->ctx->num_cu / std::max(1, d->n_batch * d->n_states);
  if (budget < 2) return;
  double e = 0.0;
  for (int k = 0; k < K; ++k) e += (double)p->nnz_ctrl[k];
  e = e / K / std::max<double>((double)p->nnz, 1.0);
  double best = 1e300;
  int bg = sh->groups, bq = 1;
  for (int g = sh->groups; g >= 1; --g) {
    const int groups = (K + g - 1) / g;
    const int q = std::min(groups, budget);
    const int passes = (groups + q - 1) / q;
    const double cost = 2.0 + passes * (1.0 + g * (1.0 + e));
    if (cost < best - 1e-9) {
      best = cost;
      bg = g;
      bq = q;
    }
  }
  sh->groups = bg;
  sh->spread = bq;
}

// Launch shape of one evaluation: one workgroup per column, the problem's
// split layout, or the dense path; then the optional spread of the backward.
static hg_status shape_for(const hg_problem* p, const hg_eval_desc* d, SweepShape* sh) {
  const int B = d->n_batch, N = d->n_steps, S = d->n_states, K = p->n_ctrl;
  const bool c128 = d->dtype == HG_C128;
  std::string why;
  *sh = SweepShape{};
  sh->parts = 1;
  sh->spread = 1;
  if (!p->dense) {
    const int parts = parts_for(p, c128);
    if (parts == 1) {
      if (!sweep_supported(p->ops, (int)p->dim, K, c128, p->ctx->lds_per_block, sh, &why))
        return fail(HG_ERR_UNSUPPORTED, why);
      sh->parts = 1;
    } else if (parts > 1) {
      if (!split_supported(p->split, K, c128, p->ctx->lds_per_block, p->ctx->num_cu, sh, &why))
        return fail(HG_ERR_UNSUPPORTED, why);
      sh->parts = parts;
      // the parts of a column wait on each other: all workgroups must be resident at once
      if ((int64_t)B * S * parts > (int64_t)p->ctx->num_cu)
        return fail(HG_ERR_UNSUPPORTED,
                    "a split evaluation needs n_batch * n_states * " + std::to_string(parts) +
                        " <= " + std::to_string(p->ctx->num_cu) + " co-resident workgroups");
    } else {
      sweep_supported(p->ops, (int)p->dim, K, c128, p->ctx->lds_per_block, sh, &why);
      return fail(HG_ERR_UNSUPPORTED, why);
    }
    sh->pure = p->ops.npure >= 3 ? 3 : 1;
    // two state columns per forward workgroup when the launch still has a
    // workgroup for every compute unit
    sh->fwd_cpw = 1;
    if (sh->parts == 1 && sh->lds_fwd2 > 0 && sh->lds_fwd2 <= p->ctx->lds_per_block && S % 2 == 0 &&
        (int64_t)B * S / 2 >= (int64_t)p->ctx->num_cu) {
      sh->fwd_cpw = 2;
      sh->lds_fwd = sh->lds_fwd2;
    }
    int wk = 1;
    for (int k = 0; k < K; ++k) wk = std::max(wk, p->ops.WK[k]);
    sh->ereal = p->ops.ereal && wk <= 2;
    sh->spread = 1;
    choose_spread(p, d, sh);
  }
  sh->n_steps = N;
  sh->n_states = S;
  sh->n_batch = B;
  return HG_OK;
}

// Checks, launch shape and buffer sizes of one evaluation (shared by the
// entry points that bring their own memory).
static hg_status eval_prepare(hg_problem* p, const hg_eval_desc* d, hg_result* results,
                              SweepShape* sh, Workspace* w) {
  hg_status st = check_desc(p, d);
  if (st != HG_OK) return st;
  if (!results) return fail(HG_ERR_INVALID_ARG, "results is NULL");
  HG_HIP(hipSetDevice(p->ctx->device));
  if ((st = shape_for(p, d, sh)) != HG_OK) return st;
  const int N = d->n_steps;
  const int ck = d->mode == HG_MODE_CHECKPOINT ? std::min(d->ckpt_every, N) : 0;
  *w = layout(p, d->n_batch, N, d->n_states, d->dtype == HG_C128, ck, d->w_int != 0.0,
              sh->spread, p->dense ? d->method : HG_METHOD_TAYLOR);
  return HG_OK;
}

}  // extern "C"

namespace hg {
hg_status eval_on_buffers(hg_problem* p, const hg_eval_desc* d, hg_result* results, double* grad,
                          hipStream_t hs, void* ws, size_t ws_bytes, void* hbuf,
                          size_t hbuf_bytes, bool build_table) {
  SweepShape sh;
  Workspace w;
  hg_status st = eval_prepare(p, d, results, &sh, &w);
  if (st != HG_OK) return st;
  if (p->dense && d->method != HG_METHOD_TAYLOR)
    return fail(HG_ERR_UNSUPPORTED, "caller-provided memory: the diagonalisation method's library "
                                    "GEMMs may allocate; use hg_eval");
  if (w.total > ws_bytes)
    return fail(HG_ERR_OUT_OF_MEMORY, "the evaluation needs " + std::to_string(w.total) +
                                          " bytes of device workspace; " +
                                          std::to_string(ws_bytes) + " are available");
  const size_t hb = host_stage_bytes(d->n_batch, d->n_steps, d->n_states, std::max(sh.parts, 1));
  if (hb > hbuf_bytes)
    return fail(HG_ERR_OUT_OF_MEMORY, "the evaluation needs " + std::to_string(hb) +
                                          " bytes of host staging; " + std::to_string(hbuf_bytes) +
                                          " are available");
  return eval_core(p, d, results, grad, hs, sh, w, (char*)ws, (char*)hbuf, build_table);
}
}  // namespace hg

extern "C" {

// Host staging of the calling thread: pinned, grown on demand and kept for the
// thread's lifetime, so a steady stream of evaluations pins no new memory.
namespace {
struct HostStage {
  char* p = nullptr;
  size_t n = 0;
  ~HostStage() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local HostStage t_stage;
}  // namespace

static hg_status eval_impl(hg_problem* p, const hg_eval_desc* d, hg_result* results, double* grad,
                           void* stream) {
  SweepShape sh;
  Workspace w;
  hg_status st = eval_prepare(p, d, results, &sh, &w);
  if (st != HG_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  // stream-ordered workspace from the device's default pool, whose release
  // threshold hg_create raises so that freed blocks stay in the pool
  char* ws = nullptr;
  if (hipMallocAsync((void**)&ws, w.total, hs) != hipSuccess)
    return fail(HG_ERR_OUT_OF_MEMORY, "workspace of " + std::to_string(w.total) + " bytes");
  struct Free {
    char* p;
    hipStream_t s;
    ~Free() {
      if (p) (void)hipFreeAsync(p, s);
    }
  } guard{ws, hs};
  const size_t hbytes = host_stage_bytes(d->n_batch, d->n_steps, d->n_states, std::max(sh.parts, 1));
  if (t_stage.n < hbytes) {
    if (t_stage.p) HG_HIP(hipHostFree(t_stage.p));
    t_stage.p = nullptr;
    t_stage.n = 0;
    const size_t want = std::max(hbytes, (size_t)1 << 20);
    HG_HIP(hipHostMalloc((void**)&t_stage.p, want, hipHostMallocDefault));
    t_stage.n = want;
  }
  return eval_core(p, d, results, grad, hs, sh, w, ws, t_stage.p, true);
}

hg_status hg_problem_create(hg_ctx* ctx, int64_t dim, int32_t n_ctrl, const hg_csr* H0,
                            const hg_csr* Hk, const double* omega_diag, hg_problem** out) {
  return guarded("hg_problem_create", [&] {
    return problem_create_impl(ctx, dim, n_ctrl, H0, Hk, omega_diag, false, out);
  });
}

hg_status hg_problem_create_dense(hg_ctx* ctx, int64_t dim, int32_t n_ctrl, const hg_csr* H0,
                                  const hg_csr* Hk, const double* omega_diag, hg_problem** out) {
  return guarded("hg_problem_create_dense", [&] {
    return problem_create_impl(ctx, dim, n_ctrl, H0, Hk, omega_diag, true, out);
  });
}

hg_status hg_plan(const double* theta, int64_t n, int32_t sigma, double tau, double u,
                  int32_t* m_out, int32_t* s_out) {
  return guarded("hg_plan", [&] { return plan_impl(theta, n, sigma, tau, u, m_out, s_out); });
}

hg_status hg_plan_rule(const double* theta, int64_t n, int32_t sigma, double tau, double u,
                       int32_t rule, int32_t* m_out, int32_t* s_out) {
  return guarded("hg_plan_rule", [&] {
    return plan_impl(theta, n, sigma, tau, u, m_out, s_out, true, rule);
  });
}

hg_status hg_eval(hg_problem* p, const hg_eval_desc* d, hg_result* results, double* grad,
                  void* stream) {
  return guarded("hg_eval", [&] { return eval_impl(p, d, results, grad, stream); });
}

hg_status hg_mem_pool_peak(hg_ctx* ctx, int32_t reset, size_t* used_high) {
  if (!ctx || !used_high) return fail(HG_ERR_INVALID_ARG, "NULL argument");
  HG_HIP(hipSetDevice(ctx->device));
  hipMemPool_t pool;
  HG_HIP(hipDeviceGetDefaultMemPool(&pool, ctx->device));
  uint64_t v = 0;
  HG_HIP(hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemHigh, &v));
  *used_high = (size_t)v;
  if (reset) {
    uint64_t z = 0;
    HG_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrUsedMemHigh, &z));
  }
  return HG_OK;
}

}  // extern "C"
