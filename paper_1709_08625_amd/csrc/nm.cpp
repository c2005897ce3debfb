// Nelder-Mead simplex minimiser (Nelder & Mead, Computer J. 7 (1965) 308-313)
// and the maximum-likelihood driver over theta = (sigma^2, ell, nu).
//
// The paper identifies theta with a derivative-free simplex search on the
// H-likelihood (Sec. 5, driver of Appendix B: initial steps 0.02, 0.04, 0.01,
// at most 200 iterations, simplex-size test).  Coefficients: reflection 1,
// expansion 2, contraction 1/2, shrink 1/2; the initial simplex is x0 and
// x0 + step_k e_k; vertices are ordered by a stable sort of their values.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <vector>

#include "../../include/hcov.h"

namespace {

struct Counter {
  hcov_objective_fn f;
  void* user;
  int n = 0, cap = 0;
  double* hist_x = nullptr;
  double* hist_f = nullptr;
  int dim = 0;
  double operator()(const std::vector<double>& x) {
    double v = f(x.data(), dim, user);
    if (hist_x && n < cap) {
      for (int i = 0; i < dim; ++i) hist_x[n * dim + i] = x[i];
      hist_f[n] = v;
    }
    ++n;
    return v;
  }
};

}  // namespace

extern "C" int hcov_nm_minimize(hcov_objective_fn f, void* user, const double* x0, const double* steps, int dim,
                                int max_evals, double size_tol, double* out_x, double* out_f, int* out_evals,
                                double* hist_x, double* hist_f) {
  if (!f || !x0 || !steps || dim < 1 || dim > 16 || max_evals < 1 || !out_x || !out_f) return HCOV_EINVAL;
  Counter F{f, user};
  F.dim = dim;
  F.cap = max_evals;
  F.hist_x = hist_x;
  F.hist_f = hist_f;
  const int d = dim;
  std::vector<std::vector<double>> S(d + 1, std::vector<double>(x0, x0 + d));
  for (int k = 0; k < d; ++k) S[k + 1][k] += steps[k];
  std::vector<double> fv(d + 1);
  for (int i = 0; i <= d && F.n < max_evals; ++i) fv[i] = F(S[i]);
  auto sort_simplex = [&]() {
    std::vector<int> idx(d + 1);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return fv[a] < fv[b]; });
    std::vector<std::vector<double>> S2(d + 1);
    std::vector<double> f2(d + 1);
    for (int i = 0; i <= d; ++i) {
      S2[i] = S[idx[i]];
      f2[i] = fv[idx[i]];
    }
    S.swap(S2);
    fv.swap(f2);
  };
  while (F.n < max_evals) {
    sort_simplex();
    std::vector<double> c(d, 0.0);
    for (int i = 0; i < d; ++i)
      for (int k = 0; k < d; ++k) c[k] += S[i][k];
    for (int k = 0; k < d; ++k) c[k] /= d;
    double size = 0.0;
    for (int i = 0; i <= d; ++i) {
      double s2 = 0.0;
      for (int k = 0; k < d; ++k) s2 += (S[i][k] - c[k]) * (S[i][k] - c[k]);
      size = std::max(size, std::sqrt(s2));
    }
    if (size < size_tol) break;
    const std::vector<double> worst = S[d];
    std::vector<double> xr(d), xe(d), xc(d);
    for (int k = 0; k < d; ++k) xr[k] = c[k] + (c[k] - worst[k]);
    double fr = F(xr);
    if (fr < fv[0]) {
      if (F.n >= max_evals) {
        S[d] = xr;
        fv[d] = fr;
        break;
      }
      for (int k = 0; k < d; ++k) xe[k] = c[k] + 2.0 * (c[k] - worst[k]);
      double fe = F(xe);
      if (fe < fr) {
        S[d] = xe;
        fv[d] = fe;
      } else {
        S[d] = xr;
        fv[d] = fr;
      }
    } else if (fr < fv[d - 1]) {
      S[d] = xr;
      fv[d] = fr;
    } else {
      if (F.n >= max_evals) break;
      if (fr < fv[d])
        for (int k = 0; k < d; ++k) xc[k] = c[k] + 0.5 * (xr[k] - c[k]);
      else
        for (int k = 0; k < d; ++k) xc[k] = c[k] + 0.5 * (worst[k] - c[k]);
      double fc = F(xc);
      if (fc < std::min(fr, fv[d])) {
        S[d] = xc;
        fv[d] = fc;
      } else {
        for (int i = 1; i <= d; ++i) {
          if (F.n >= max_evals) break;
          for (int k = 0; k < d; ++k) S[i][k] = S[0][k] + 0.5 * (S[i][k] - S[0][k]);
          fv[i] = F(S[i]);
        }
      }
    }
  }
  int b = int(std::min_element(fv.begin(), fv.end()) - fv.begin());
  for (int k = 0; k < d; ++k) out_x[k] = S[b][k];
  *out_f = fv[b];
  if (out_evals) *out_evals = F.n;
  return HCOV_OK;
}

namespace {
struct FitCtx {
  hcov_ctx* ctx;
  const double* z;
  int where;
  double nugget;
  int last_rc;
};
double neg_loglik(const double* x, int dim, void* user) {
  (void)dim;
  FitCtx* F = static_cast<FitCtx*>(user);
  hcov_theta th{x[0], x[1], x[2], F->nugget};
  if (!(x[0] > 0) || !(x[1] > 0) || !(x[2] > 0)) return std::numeric_limits<double>::infinity();
  int rc = hcov_set_theta(F->ctx, th);
  double ll = 0;
  if (rc == HCOV_OK) rc = hcov_loglik(F->ctx, F->z, F->where, &ll, nullptr, nullptr);
  if (rc != HCOV_OK) {
    if (rc == HCOV_EDEVICE) F->last_rc = rc;
    return std::numeric_limits<double>::infinity();
  }
  return -ll;
}
}  // namespace

extern "C" int hcov_fit(hcov_ctx* ctx, const double* z, int where, const double* theta0, const double* steps,
                        double nugget, int max_evals, double size_tol, double* out_theta, double* out_ll,
                        int* out_evals, double* hist_theta, double* hist_negll) {
  if (!ctx || !z || !theta0 || !out_theta || !out_ll) return HCOV_EINVAL;
  const double def_steps[3] = {0.01, 0.04, 0.02};   // (sigma^2, ell, nu) as in the paper's driver
  FitCtx F{ctx, z, where, nugget, HCOV_OK};
  double fbest = 0;
  int rc = hcov_nm_minimize(neg_loglik, &F, theta0, steps ? steps : def_steps, 3, max_evals, size_tol, out_theta,
                            &fbest, out_evals, hist_theta, hist_negll);
  if (rc) return rc;
  if (F.last_rc) return F.last_rc;
  *out_ll = -fbest;
  return HCOV_OK;
}
