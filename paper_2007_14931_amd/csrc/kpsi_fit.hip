// Host-side fit driver of libkpsi: a variable-metric minimiser in the style of MINUIT's
// MIGRAD and a HESSE covariance, on top of kpsi_nll / kpsi_nll_and_grad.
//
// The paper's fit loop steps the parameters on the host and evaluates the PDF/NLL on the
// device (Introduction); with more than 60 free parameters (text after Eq. 12) the
// gradient is the expensive part.  Two gradient modes are provided:
//   analytic: one kpsi_nll_and_grad call (the device adjoint) per gradient;
//   finite differences: 2 P kpsi_nll calls per gradient (central differences), the
//   plain form used for comparison.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kpsi_internal.h"

namespace {

struct Problem {
  kpsi_ctx* c;
  std::vector<double> full;     // full parameter vector (fixed entries kept)
  std::vector<int> idx;         // free indices
  bool analytic;
  double h_rel;
  int64_t n_nll = 0, n_grad = 0;
  int64_t max_calls;
  std::vector<double> gfull;

  // Limits (MINUIT's transformations): the minimiser works on an internal variable u per free
  // parameter; a parameter limited on both sides is lo + (hi - lo)(sin u + 1)/2, one limited
  // below is lo - 1 + sqrt(u^2 + 1), one limited above is hi + 1 - sqrt(u^2 + 1).
  std::vector<int> kind;        // per free parameter: 0 none, 1 both, 2 below, 3 above
  std::vector<double> lo, hi;

  int n() const { return (int)idx.size(); }
  double ext(int i, double u) const {
    switch (kind.empty() ? 0 : kind[i]) {
      case 1: return lo[i] + 0.5 * (hi[i] - lo[i]) * (std::sin(u) + 1.0);
      case 2: return lo[i] - 1.0 + std::sqrt(u * u + 1.0);
      case 3: return hi[i] + 1.0 - std::sqrt(u * u + 1.0);
      default: return u;
    }
  }
  double dext(int i, double u) const {   // d ext / d u
    switch (kind.empty() ? 0 : kind[i]) {
      case 1: return 0.5 * (hi[i] - lo[i]) * std::cos(u);
      case 2: return u / std::sqrt(u * u + 1.0);
      case 3: return -u / std::sqrt(u * u + 1.0);
      default: return 1.0;
    }
  }
  double intl(int i, double x) const {   // the internal value of an external one inside its limits
    switch (kind.empty() ? 0 : kind[i]) {
      case 1: return std::asin(2.0 * (x - lo[i]) / (hi[i] - lo[i]) - 1.0);
      case 2: { const double t = x - lo[i] + 1.0; return std::sqrt(t * t - 1.0); }
      case 3: { const double t = hi[i] - x + 1.0; return std::sqrt(t * t - 1.0); }
      default: return x;
    }
  }
  void put(const std::vector<double>& x) { for (int i = 0; i < n(); ++i) full[idx[i]] = ext(i, x[i]); }
  bool budget() const { return n_nll + n_grad < max_calls; }

  // f(x); +inf when the point is rejected (non-finite density, unphysical mass or width)
  double f(const std::vector<double>& x) {
    put(x);
    double v = 0.0;
    ++n_nll;
    kpsi_status st = kpsi_nll(c, full.data(), &v);
    if (st == KPSI_OK && std::isfinite(v)) return v;
    if (st == KPSI_E_NONFINITE || st == KPSI_E_ARG) return INFINITY;
    return NAN;   // hard error (device failure): caller stops
  }
  double step(int i, const std::vector<double>& x) const { return h_rel * (1.0 + std::fabs(x[i])); }

  // f and gradient at x; g2 receives a diagonal curvature estimate when available
  double fg(const std::vector<double>& x, std::vector<double>& g, std::vector<double>* g2) {
    g.assign(n(), 0.0);
    if (analytic) {
      put(x);
      gfull.assign(full.size(), 0.0);
      double v = 0.0;
      ++n_grad;
      kpsi_status st = kpsi_nll_and_grad(c, full.data(), &v, gfull.data());
      if (st == KPSI_E_NONFINITE || st == KPSI_E_ARG) return INFINITY;
      if (st != KPSI_OK) return NAN;
      for (int i = 0; i < n(); ++i) g[i] = gfull[idx[i]] * dext(i, x[i]);
      return v;
    }
    const double f0 = f(x);
    if (!std::isfinite(f0)) return f0;
    std::vector<double> xp = x;
    for (int i = 0; i < n(); ++i) {
      const double h = step(i, x);
      xp[i] = x[i] + h;
      const double fp = f(xp);
      xp[i] = x[i] - h;
      const double fm = f(xp);
      xp[i] = x[i];
      if (!std::isfinite(fp) || !std::isfinite(fm)) return std::isnan(fp) || std::isnan(fm) ? NAN : INFINITY;
      g[i] = (fp - fm) / (2.0 * h);
      if (g2) (*g2)[i] = (fp - 2.0 * f0 + fm) / (h * h);
    }
    return f0;
  }
};

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// Diagonal curvature from gradient differences (analytic mode).
bool curvature(Problem& p, const std::vector<double>& x, std::vector<double>& g2) {
  std::vector<double> xp = x, gp, gm;
  for (int i = 0; i < p.n(); ++i) {
    const double h = p.step(i, x) * 100.0;
    xp[i] = x[i] + h;
    double a = p.fg(xp, gp, nullptr);
    xp[i] = x[i] - h;
    double b = p.fg(xp, gm, nullptr);
    xp[i] = x[i];
    if (!std::isfinite(a) || !std::isfinite(b)) { g2[i] = 1.0; continue; }
    g2[i] = (gp[i] - gm[i]) / (2.0 * h);
  }
  return true;
}

// Cholesky inverse of a symmetric positive-definite matrix (row-major, n x n).
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(A.size(), 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = s / L[j * n + j];
    }
  }
  // inverse of L, then A^-1 = L^-T L^-1
  std::vector<double> Li(A.size(), 0.0);
  for (int i = 0; i < n; ++i) {
    Li[i * n + i] = 1.0 / L[i * n + i];
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = -s / L[i * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Li[k * n + i] * Li[k * n + j];
      A[i * n + j] = A[j * n + i] = s;
    }
  return true;
}

// Inverse of H + tau I for the smallest tau in {0, 1e-6, 1e-5, ..., 10} x max |H_ii| for which the
// shifted matrix is positive definite (MINUIT's positive-definite forcing); false if none is.
bool forced_pd_inverse(const std::vector<double>& H, int n, std::vector<double>& inv) {
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(H[(size_t)i * n + i]));
  if (!(dmax > 0.0) || !std::isfinite(dmax)) dmax = 1.0;
  for (int k = -7; k <= 1; ++k) {
    const double tau = k < -6 ? 0.0 : dmax * std::pow(10.0, k);
    inv = H;
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] += tau;
    if (spd_inverse(inv, n)) return true;
  }
  return false;
}

kpsi_status hesse_impl(Problem& p, const std::vector<double>& x, double up, double* cov, bool* pd,
                       std::vector<double>* hraw = nullptr) {
  const int n = p.n();
  std::vector<double> H((size_t)n * n, 0.0);
  if (p.analytic) {
    std::vector<double> xp = x, gp, gm;
    for (int j = 0; j < n; ++j) {
      const double h = p.step(j, x) * 10.0;
      xp[j] = x[j] + h;
      double a = p.fg(xp, gp, nullptr);
      xp[j] = x[j] - h;
      double b = p.fg(xp, gm, nullptr);
      xp[j] = x[j];
      if (std::isnan(a) || std::isnan(b)) return KPSI_E_HIP;
      for (int i = 0; i < n; ++i) H[i * n + j] = (gp[i] - gm[i]) / (2.0 * h);
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) H[i * n + j] = H[j * n + i] = 0.5 * (H[i * n + j] + H[j * n + i]);
  } else {
    const double f0 = p.f(x);
    if (std::isnan(f0)) return KPSI_E_HIP;
    std::vector<double> xp = x, hs(n);
    for (int i = 0; i < n; ++i) hs[i] = p.step(i, x) * 10.0;
    for (int i = 0; i < n; ++i) {
      xp[i] = x[i] + hs[i];
      const double fp = p.f(xp);
      xp[i] = x[i] - hs[i];
      const double fm = p.f(xp);
      xp[i] = x[i];
      H[i * n + i] = (fp - 2.0 * f0 + fm) / (hs[i] * hs[i]);
      for (int j = 0; j < i; ++j) {
        double v[4];
        const int sg[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
        for (int k = 0; k < 4; ++k) {
          xp[i] = x[i] + sg[k][0] * hs[i];
          xp[j] = x[j] + sg[k][1] * hs[j];
          v[k] = p.f(xp);
        }
        xp[i] = x[i];
        xp[j] = x[j];
        H[i * n + j] = H[j * n + i] = (v[0] - v[1] - v[2] + v[3]) / (4.0 * hs[i] * hs[j]);
      }
    }
  }
  // covariance of the parameters for an NLL scale with error definition `up`: 2 up H^-1
  if (hraw) *hraw = H;
  *pd = spd_inverse(H, n);
  if (cov) for (size_t k = 0; k < H.size(); ++k) cov[k] = *pd ? 2.0 * up * H[k] : NAN;
  return KPSI_OK;
}

kpsi_status setup(Problem& p, kpsi_ctx* c, const double* params, const int* free_mask, const kpsi_fit_options* o,
                  const double* lower = nullptr, const double* upper = nullptr) {
  int np = 0;
  kpsi_status st = kpsi_n_params(c, &np);
  if (st) return st;
  p.c = c;
  p.full.assign(params, params + np);
  p.idx.clear();
  for (int i = 0; i < np; ++i) if (free_mask[i]) p.idx.push_back(i);
  p.kind.clear();
  if (lower || upper) {
    const int n = p.n();
    p.kind.assign(n, 0);
    p.lo.assign(n, 0.0);
    p.hi.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
      const int k = p.idx[i];
      const double a = lower ? lower[k] : NAN, b = upper ? upper[k] : NAN;
      const bool la = std::isfinite(a), lb = std::isfinite(b);
      char msg[160];
      if (la && lb && !(a < b)) {
        snprintf(msg, sizeof msg, "parameter %d: lower limit %g is not below the upper limit %g", k, a, b);
        return kpsi::set_error(c, KPSI_E_ARG, msg);
      }
      p.kind[i] = la && lb ? 1 : (la ? 2 : (lb ? 3 : 0));
      p.lo[i] = a;
      p.hi[i] = b;
      // the start must lie strictly inside its limits
      if ((la && !(params[k] > a)) || (lb && !(params[k] < b))) {
        snprintf(msg, sizeof msg, "parameter %d: start %g is not strictly inside its limits (%g, %g)", k, params[k],
                 a, b);
        return kpsi::set_error(c, KPSI_E_ARG, msg);
      }
    }
  }
  p.analytic = o->gradient != 0;
  p.h_rel = o->fd_rel_step > 0.0 ? o->fd_rel_step : 1e-5;
  p.max_calls = o->max_calls > 0 ? o->max_calls : 100000;
  return p.idx.empty() ? KPSI_E_ARG : KPSI_OK;
}

}  // namespace

extern "C" {

kpsi_status kpsi_fit_default_options(kpsi_fit_options* o) {
  if (!o) return KPSI_E_ARG;
  o->max_calls = 100000;
  o->tolerance = 0.1;
  o->up = 1.0;
  o->gradient = 1;
  o->fd_rel_step = 1e-5;
  o->hesse = 1;
  return KPSI_OK;
}

static kpsi_status migrad_impl(kpsi_ctx* c, double* params, const int* free_mask, const double* lower,
                               const double* upper, const kpsi_fit_options* o, kpsi_fit_result* r, double* cov) {
  if (!c || !params || !free_mask || !o || !r) return KPSI_E_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  Problem p;
  kpsi_status st = setup(p, c, params, free_mask, o, lower, upper);
  if (st) return st;
  const int n = p.n();
  const double up = o->up > 0.0 ? o->up : 1.0;
  const double edm_target = 0.002 * (o->tolerance > 0.0 ? o->tolerance : 0.1) * up;
  std::memset(r, 0, sizeof *r);
  std::vector<double> x(n), g, g2(n, 0.0), V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) x[i] = p.intl(i, p.full[p.idx[i]]);
  double fx = p.fg(x, g, p.analytic ? nullptr : &g2);
  if (!std::isfinite(fx)) { r->status = 4; r->fmin = fx; return std::isnan(fx) ? KPSI_E_HIP : KPSI_E_NONFINITE; }
  if (p.analytic) curvature(p, x, g2);
  auto seed_metric = [&]() {
    std::fill(V.begin(), V.end(), 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = g2[i] > 0.0 ? 1.0 / g2[i] : 1.0;
  };
  seed_metric();
  std::vector<double> d(n), x1(n), g1, s(n), y(n), Vy(n), Hm;
  int it = 0, status = 1, restarts = 0;
  double edm = 0.0;
  bool have_cov = false;
restart:
  for (; p.budget(); ++it) {
    // Newton step in the current metric and the expected distance to the minimum
    for (int i = 0; i < n; ++i) {
      double a = 0.0;
      for (int j = 0; j < n; ++j) a += V[(size_t)i * n + j] * g[j];
      d[i] = -a;
    }
    double gd = dot(g, d);
    edm = -0.5 * gd;
    if (edm < edm_target) { status = 0; break; }
    if (gd >= 0.0) {   // metric lost positive definiteness: restart from the diagonal
      seed_metric();
      for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int j = 0; j < n; ++j) a += V[(size_t)i * n + j] * g[j];
        d[i] = -a;
      }
      gd = dot(g, d);
    }
    // line search: full step, then parabolic backtracking (Armijo condition)
    double alpha = 1.0, f1 = INFINITY;
    bool ok = false;
    for (int ls = 0; ls < 12 && p.budget(); ++ls) {
      for (int i = 0; i < n; ++i) x1[i] = x[i] + alpha * d[i];
      f1 = p.f(x1);
      if (std::isnan(f1)) { r->status = 4; return KPSI_E_HIP; }
      if (f1 <= fx + 1e-4 * alpha * gd) { ok = true; break; }
      double an = std::isfinite(f1) ? -gd * alpha * alpha / (2.0 * (f1 - fx - alpha * gd)) : 0.1 * alpha;
      alpha = std::min(0.5 * alpha, std::max(0.1 * alpha, an));
    }
    if (!ok) { status = 2; break; }
    double f1g = p.fg(x1, g1, p.analytic ? nullptr : &g2);
    if (std::isnan(f1g)) { r->status = 4; return KPSI_E_HIP; }
    if (!std::isfinite(f1g)) { status = 2; break; }
    for (int i = 0; i < n; ++i) { s[i] = x1[i] - x[i]; y[i] = g1[i] - g[i]; }
    const double ys = dot(y, s);
    if (ys > 1e-300) {
      // BFGS update of the inverse metric: V <- V + ((s.y + y.Vy)/(s.y)^2) s s^T - (Vy s^T + s (Vy)^T)/(s.y)
      for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int j = 0; j < n; ++j) a += V[(size_t)i * n + j] * y[j];
        Vy[i] = a;
      }
      const double yVy = dot(y, Vy);
      const double c1 = (ys + yVy) / (ys * ys);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          V[(size_t)i * n + j] += c1 * s[i] * s[j] - (Vy[i] * s[j] + s[i] * Vy[j]) / ys;
    }
    x = x1;
    g = g1;
    fx = f1g;
  }
  if (o->hesse && (status == 0 || status == 2)) {
    // MINUIT's check: the variable-metric estimate can understate the distance to the
    // minimum; recompute EDM with the numerical Hessian and continue from it if needed.
    bool pd = false;
    Hm.assign((size_t)n * n, 0.0);
    std::vector<double> Hraw;
    st = hesse_impl(p, x, up, Hm.data(), &pd, &Hraw);
    if (st) return st;
    if (pd) {
      have_cov = true;
      double e2 = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) e2 += g[i] * Hm[(size_t)i * n + j] * g[j];
      e2 *= 0.5 / (2.0 * up);   // Hm = 2 up H^-1
      edm = e2;
      if (e2 < edm_target) status = 0;
      else if (restarts < 3 && p.budget()) {
        ++restarts;
        for (size_t k = 0; k < V.size(); ++k) V[k] = Hm[k] / (2.0 * up);
        status = 1;
        have_cov = false;
        goto restart;
      }
    } else {
      // The numerical Hessian is not positive definite.  The variable-metric estimate may have
      // stopped the search early (it can understate the distance to the minimum far from it):
      // with the Hessian forced positive definite, continue if the distance it predicts is
      // above the target; otherwise (a saddle or a flat direction) report status 3.
      std::vector<double> Vf;
      status = 3;
      if (restarts < 3 && p.budget() && forced_pd_inverse(Hraw, n, Vf)) {
        double e2 = 0.0;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) e2 += g[i] * Vf[(size_t)i * n + j] * g[j];
        edm = 0.5 * e2;
        if (edm >= edm_target) {
          ++restarts;
          V = Vf;
          status = 1;
          goto restart;
        }
      }
    }
  }
  r->fmin = fx;
  r->edm = edm;
  r->n_iter = it;
  r->status = status;
  for (int i = 0; i < n; ++i) params[p.idx[i]] = p.ext(i, x[i]);
  if (o->hesse) {
    if (have_cov) {
      if (cov) std::copy(Hm.begin(), Hm.end(), cov);
    } else {
      bool pd = false;
      st = hesse_impl(p, x, up, cov, &pd);
      if (st) return st;
      if (!pd && r->status == 0) r->status = 3;
    }
  } else if (cov) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) cov[(size_t)i * n + j] = 2.0 * up * V[(size_t)i * n + j];
  }
  // limited parameters: the internal covariance mapped to the external parameters with the
  // derivatives of the transformations at the minimum (first order, as MINUIT reports it)
  if (cov && !p.kind.empty()) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) cov[(size_t)i * n + j] *= p.dext(i, x[i]) * p.dext(j, x[j]);
  }
  r->n_nll = p.n_nll;
  r->n_grad = p.n_grad;
  r->wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return KPSI_OK;
}

kpsi_status kpsi_migrad(kpsi_ctx* c, double* params, const int* free_mask, const kpsi_fit_options* o,
                        kpsi_fit_result* r, double* cov) {
  return migrad_impl(c, params, free_mask, nullptr, nullptr, o, r, cov);
}

kpsi_status kpsi_migrad_limited(kpsi_ctx* c, double* params, const int* free_mask, const double* lower,
                                const double* upper, const kpsi_fit_options* o, kpsi_fit_result* r, double* cov) {
  return migrad_impl(c, params, free_mask, lower, upper, o, r, cov);
}

kpsi_status kpsi_hesse(kpsi_ctx* c, const double* params, const int* free_mask, const kpsi_fit_options* o,
                       double* cov, kpsi_fit_result* r) {
  if (!c || !params || !free_mask || !o || !cov) return KPSI_E_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  Problem p;
  kpsi_status st = setup(p, c, params, free_mask, o);
  if (st) return st;
  std::vector<double> x(p.n());
  for (int i = 0; i < p.n(); ++i) x[i] = p.full[p.idx[i]];
  bool pd = false;
  st = hesse_impl(p, x, o->up > 0.0 ? o->up : 1.0, cov, &pd);
  if (r) {
    std::memset(r, 0, sizeof *r);
    r->status = pd ? 0 : 3;
    r->n_nll = p.n_nll;
    r->n_grad = p.n_grad;
    r->wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // extern "C"
