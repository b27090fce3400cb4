// Host planner: the error bound E_A(m, s) of App. C and the (m, s) selection
// rule of Sec. III.B, in FP64.  Built with -ffp-contract=off so every product
// and sum is rounded exactly as written.
//
//   R_m(x)  = sum_{q>m} x^q/q!                          (App. C.1)
//   trunc   = sR (1 - (sR)^s) / (1 - sR), R = R_m(theta/s)   (App. C.1, eq. truncation)
//   u'      = 2 sqrt(2) u / (1 - 2u),  gamma_n = n u'/(1 - n u')  (App. C.2)
//   beta    = sum_{k=0..m} gamma_{k(sigma+2)+m+2} (theta/s)^k / k!   (App. C.2, eq. B23)
//   alpha   = 1 + R                                      (App. C.3)
//   E_A     = trunc + (alpha+beta)^s - alpha^s           (App. C, eq. overallupperbound)
//
// Readings: sR >= 1 is infeasible; gamma_n is infinite once n u' >= 1; the
// tail is summed directly until a term drops below 1e-18 of the sum; the
// rounding part is evaluated as alpha^s expm1(s log1p(beta/alpha)); s runs
// 1, 2, ... up to floor(tau / gamma_3), m runs 1..60, first hit wins.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

namespace hg {

namespace {

double u_prime(double u) { return 2.0 * std::sqrt(2.0) * u / (1.0 - 2.0 * u); }

double gamma_n(int64_t n, double up) {
  double nu = (double)n * up;
  if (nu >= 1.0) return std::numeric_limits<double>::infinity();
  return nu / (1.0 - nu);
}

double taylor_tail(double x, int m) {
  if (x == 0.0) return 0.0;
  double t = 1.0;
  for (int q = 1; q <= m + 1; ++q) t = t * x / (double)q;
  double total = t;
  int q = m + 1;
  for (;;) {
    q += 1;
    t = t * x / (double)q;
    total += t;
    if (!(t >= 1e-18 * total) || std::isinf(total)) break;
  }
  return total;
}

// beta of App. C.2 (eq. B23) at scaled norm x.
double beta_of(double x, int m, int sigma, double up) {
  double beta = 0.0;
  double t = 1.0;
  for (int k = 0; k <= m; ++k) {
    if (k > 0) t = t * x / (double)k;
    beta += gamma_n((int64_t)k * (sigma + 2) + m + 2, up) * t;
  }
  return beta;
}

}  // namespace

double error_bound(double theta, int m, int s, int sigma, double u) {
  const double x = theta / (double)s;
  const double R = taylor_tail(x, m);
  const double sR = (double)s * R;
  if (!(sR < 1.0)) return std::numeric_limits<double>::infinity();
  const double trunc = sR * (1.0 - std::pow(sR, (double)s)) / (1.0 - sR);
  const double up = u_prime(u);
  const double alpha = 1.0 + R;
  const double beta = beta_of(x, m, sigma, up);
  if (std::isinf(beta)) return std::numeric_limits<double>::infinity();
  const double rnd = std::pow(alpha, (double)s) * std::expm1((double)s * std::log1p(beta / alpha));
  return trunc + rnd;
}

// Smallest s, then smallest m (Sec. III.B).  The inner scan over m may stop
// early once s*beta(m) > 2 tau: the rounding part (alpha+beta)^s - alpha^s is at
// least s*beta and beta grows with m, so no larger m can satisfy the bound
// (the factor 2 keeps the shortcut clear of rounding in the comparison).
// Returns 0 on success, 1 if no (m, s) exists, 2 if one might exist only
// beyond s = kSCap (a single step would then cost more than 60*kSCap products).
static constexpr int64_t kSCap = 4096;
static int select_one(double theta, int sigma, double tau, double u, int32_t* m_out,
                      int32_t* s_out) {
  const double up = u_prime(u);
  const double g3 = gamma_n(3, up);
  int64_t s_lim = (int64_t)(tau / g3);
  if (s_lim < 1) s_lim = 1;
  const bool capped = s_lim > kSCap;
  if (capped) s_lim = kSCap;
  for (int64_t s = 1; s <= s_lim; ++s) {
    const double x = theta / (double)s;
    for (int m = 1; m <= 60; ++m) {
      if (error_bound(theta, m, (int)s, sigma, u) <= tau) {
        *m_out = m;
        *s_out = (int32_t)s;
        return 0;
      }
      if ((double)s * beta_of(x, m, sigma, up) > 2.0 * tau) break;
    }
  }
  return capped ? 2 : 1;
}

// Fewest products mu = m s under the same bound (ties: the smaller s).  For
// each s the smallest feasible m is the cheapest; s beyond the best mu found
// cannot win.  Same return codes as select_one.
static int select_one_min_mu(double theta, int sigma, double tau, double u, int32_t* m_out,
                             int32_t* s_out) {
  const double up = u_prime(u);
  const double g3 = gamma_n(3, up);
  int64_t s_lim = (int64_t)(tau / g3);
  if (s_lim < 1) s_lim = 1;
  const bool capped = s_lim > kSCap;
  if (capped) s_lim = kSCap;
  int64_t best = -1;
  for (int64_t s = 1; s <= s_lim; ++s) {
    if (best >= 0 && s > best) break;
    const double x = theta / (double)s;
    for (int m = 1; m <= 60; ++m) {
      if (error_bound(theta, m, (int)s, sigma, u) <= tau) {
        if (best < 0 || (int64_t)m * s < best) {
          best = (int64_t)m * s;
          *m_out = m;
          *s_out = (int32_t)s;
        }
        break;
      }
      if ((double)s * beta_of(x, m, sigma, up) > 2.0 * tau) break;
    }
  }
  if (best >= 0) return 0;
  return capped ? 2 : 1;
}

namespace {

bool near(double a, double b) { return b >= 0.0 && std::fabs(a - b) <= 1e-12 * std::max(a, b); }

// Feasibility thresholds for fixed (sigma, tau, u): th[s][m] is the largest
// norm theta with E_A(m, s, theta) <= tau (negative if none), found by
// bisection on the same floating-point function the direct search uses.
// Because E_A grows with theta, "E_A(m, s, theta) <= tau" is "theta <= th[s][m]"
// except within rounding noise of the threshold; lookups that land within
// 1e-12 (relative) of any deciding threshold fall back to the direct search,
// so every decision equals the direct search's.
struct Thresholds {
  int sigma = 0;
  double tau = 0.0, u = 0.0;
  std::vector<std::array<double, 61>> th;  // index s (1-based), m (1..60)
  std::vector<double> smax;                // max_m th[s][m]
  std::vector<std::pair<double, int64_t>> sorted;  // every threshold >= 0 with its s, ascending
  int64_t s_lim = 0;
  bool capped = false;

  double threshold(int m, int s) const {
    if (!(error_bound(0.0, m, s, sigma, u) <= tau)) return -1.0;
    double lo = 0.0, hi = 1.0;
    while (error_bound(hi, m, s, sigma, u) <= tau) {
      lo = hi;
      hi *= 2.0;
      if (hi > 1e12) return lo;
    }
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (error_bound(mid, m, s, sigma, u) <= tau) lo = mid; else hi = mid;
    }
    return lo;
  }

  // make sure rows 1..s exist
  void extend(int64_t s) {
    if (th.empty()) {
      th.resize(1);
      smax.assign(1, -1.0);
    }
    while ((int64_t)th.size() <= s) {
      const int ss = (int)th.size();
      std::array<double, 61> row;
      row[0] = -1.0;
      double mx = -1.0;
      const double up = u_prime(u);
      for (int m = 1; m <= 60; ++m) {
        // beta at theta = 0 is gamma_{m+2}; once s*gamma_{m+2} > 2 tau no larger m is feasible
        if ((double)ss * gamma_n(m + 2, up) > 2.0 * tau) {
          for (int mm = m; mm <= 60; ++mm) row[mm] = -1.0;
          break;
        }
        row[m] = threshold(m, ss);
        mx = std::max(mx, row[m]);
      }
      th.push_back(row);
      smax.push_back(mx);
      const size_t old = sorted.size();
      for (int m = 1; m <= 60; ++m)
        if (row[m] >= 0.0) sorted.emplace_back(row[m], (int64_t)ss);
      std::sort(sorted.begin() + old, sorted.end());
      std::inplace_merge(sorted.begin(), sorted.begin() + old, sorted.end());
    }
  }

  // Is theta within rounding noise (near) of any threshold of rows 1..s_max?
  // Every b with near(t, b) lies in [t (1 - 2e-12), t (1 + 2e-12)], so only
  // that slice of the sorted thresholds is tested, with near() itself.
  bool near_any(double t, int64_t s_max) const {
    auto it = std::lower_bound(sorted.begin(), sorted.end(),
                               std::make_pair(t * (1.0 - 2e-12), std::numeric_limits<int64_t>::min()));
    for (; it != sorted.end() && it->first <= t * (1.0 + 2e-12); ++it)
      if (it->second <= s_max && near(t, it->first)) return true;
    return false;
  }
};

std::mutex g_tab_mu;
std::map<std::tuple<int, double, double>, std::shared_ptr<Thresholds>> g_tabs;

std::shared_ptr<Thresholds> table_for(int sigma, double tau, double u) {
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto key = std::make_tuple(sigma, tau, u);
  auto it = g_tabs.find(key);
  if (it != g_tabs.end()) return it->second;
  auto t = std::make_shared<Thresholds>();
  t->sigma = sigma;
  t->tau = tau;
  t->u = u;
  const double g3 = gamma_n(3, u_prime(u));
  t->s_lim = std::max<int64_t>(1, (int64_t)(tau / g3));
  t->capped = t->s_lim > kSCap;
  if (t->capped) t->s_lim = kSCap;
  g_tabs[key] = t;
  return t;
}

}  // namespace

int plan_steps(const double* theta, int64_t n, int sigma, double tau, double u, int32_t* m_out,
               int32_t* s_out, int64_t* fail_index, bool build_table, int rule) {
  std::shared_ptr<Thresholds> tab;
  if (build_table) {
    tab = table_for(sigma, tau, u);
  } else {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tabs.find(std::make_tuple(sigma, tau, u));
    if (it != g_tabs.end()) tab = it->second;
  }
  auto direct = rule == 1 ? select_one_min_mu : select_one;
  if (!tab) {  // direct search only
    for (int64_t i = 0; i < n; ++i) {
      const int rc = direct(theta[i], sigma, tau, u, &m_out[i], &s_out[i]);
      if (rc != 0) {
        *fail_index = i;
        return rc;
      }
    }
    return 0;
  }
  std::lock_guard<std::mutex> lk(g_tab_mu);  // the table grows lazily
  if (rule == 1) {
    for (int64_t i = 0; i < n; ++i) {
      const double t = theta[i];
      int64_t best = -1;
      int bm = 0;
      int64_t bs = 0;
      bool exact = true;
      for (int64_t s = 1; s <= tab->s_lim; ++s) {
        if (best >= 0 && s > best) break;
        if (!build_table && (int64_t)tab->th.size() <= s) {
          exact = false;
          break;
        }
        tab->extend(s);
        if (tab->near_any(t, s)) {
          exact = false;
          break;
        }
        if (t <= tab->smax[s]) {
          int m = 1;
          while (m <= 60 && !(t <= tab->th[s][m])) ++m;
          if (m <= 60 && (best < 0 || (int64_t)m * s < best)) {
            best = (int64_t)m * s;
            bm = m;
            bs = s;
          }
        }
      }
      if (exact && best >= 0) {
        m_out[i] = bm;
        s_out[i] = (int32_t)bs;
        continue;
      }
      const int rc = select_one_min_mu(t, sigma, tau, u, &m_out[i], &s_out[i]);
      if (rc != 0) {
        *fail_index = i;
        return rc;
      }
    }
    return 0;
  }
  for (int64_t i = 0; i < n; ++i) {
    const double t = theta[i];
    // smallest s whose best threshold admits t, growing the table as needed
    // (without build_table, only as far as it already reaches)
    int64_t s = 1;
    bool found = false;
    bool beyond = false;
    for (; s <= tab->s_lim; ++s) {
      if (!build_table && (int64_t)tab->th.size() <= s) {
        beyond = true;
        break;
      }
      tab->extend(s);
      if (t <= tab->smax[s]) {
        found = true;
        break;
      }
    }
    bool exact = found && !beyond;
    int m = 0;
    if (found) {
      for (m = 1; m <= 60; ++m)
        if (t <= tab->th[s][m]) break;
      // decisions made close to a threshold are re-taken by the direct search
      if (exact && tab->near_any(t, s)) exact = false;
    }
    if (exact) {
      m_out[i] = m;
      s_out[i] = (int32_t)s;
      continue;
    }
    const int rc = select_one(t, sigma, tau, u, &m_out[i], &s_out[i]);
    if (rc != 0) {
      *fail_index = i;
      return rc;
    }
  }
  return 0;
}

}  // namespace hg
