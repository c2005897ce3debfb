// Matérn covariance of Eq. (3) (Sec. 2.1) on the device:
//   C(h) = sigma^2 / (2^(nu-1) Gamma(nu)) * x^nu * K_nu(x),   x = h / ell,
// with C(0) = sigma^2.  K_nu is evaluated by
//   * the elementary closed forms for nu = 1/2, 3/2, 5/2 (Sec. 2.1 names the
//     nu = 1/2 case the exponential kernel);
//   * Temme's series (N. M. Temme, J. Comput. Phys. 19 (1975) 324-337) for
//     K_mu and K_{mu+1}, |mu| <= 1/2, when x <= 2, followed by the upward
//     recurrence K_{m+1}(x) = (2m/x) K_m(x) + K_{m-1}(x) (DLMF 10.29.1);
//   * for x > 2, the integral e^x K_nu(x) = int_0^inf exp(-x (cosh t - 1))
//     cosh(nu t) dt (DLMF 10.32.9) by the trapezoidal rule with step
//     0.25/sqrt(x), whose error decays like exp(-2 pi d / h) for an integrand
//     analytic in a strip of half-width d; cosh t - 1 = 2 sinh^2(t/2) avoids
//     cancellation, and sinh / cosh along the nodes follow from the addition
//     theorems.
// The nu-only constants (Gamma_1, Gamma_2, Gamma(1 +- mu), the normalisation)
// are computed once per theta on the host (see hcov.cpp).
#pragma once

#include "common.h"

namespace hc {

__device__ __forceinline__ double matern_closed(double x, const MaternParams& P) {
  double e = exp(-x);
  if (P.kind == 1) return P.sigma2 * e;
  if (P.kind == 2) return P.sigma2 * (1.0 + x) * e;
  return P.sigma2 * (1.0 + x + x * x * (1.0 / 3.0)) * e;
}

// x^nu K_nu(x) for 0 < x <= 2 via Temme's series and the recurrence.
__device__ __noinline__ double xnu_knu_series(double x, const MaternParams& P) {
  const double mu = P.mu;
  const double lnx2 = -log(0.5 * x);          // ln(2/x)
  const double sig = mu * lnx2;
  const double ep = exp(sig);                 // (x/2)^(-mu)
  const double em = 1.0 / ep;                 // (x/2)^(mu)
  const double coshs = 0.5 * (ep + em);
  double shs;                                 // sinh(sig)/sig
  if (fabs(sig) < 1e-3) {
    double s2 = sig * sig;
    shs = 1.0 + s2 * (1.0 / 6.0) * (1.0 + s2 * (1.0 / 20.0));
  } else {
    shs = 0.5 * (ep - em) / sig;
  }
  double f = P.mupi * (coshs * P.g1 + shs * lnx2 * P.g2);
  double p = 0.5 * ep * P.gp;
  double q = 0.5 * em * P.gm;
  double c = 1.0;
  const double y = 0.25 * x * x;
  double s0 = f;       // sum c_k f_k      -> K_mu
  double s1 = p;       // sum c_k h_k      -> x/2 K_{mu+1}
  const double mu2 = mu * mu;
  for (int k = 1; k < 80; ++k) {
    double dk = double(k);
    f = (dk * f + p + q) / (dk * dk - mu2);
    p = p / (dk - mu);
    q = q / (dk + mu);
    c = c * y / dk;
    double t0 = c * f;
    double h = p - dk * f;
    s0 += t0;
    s1 += c * h;
    if (fabs(t0) < 1e-17 * fabs(s0) && fabs(c * h) < 1e-17 * fabs(s1)) break;
  }
  double k0 = s0;
  double k1 = s1 * 2.0 / x;
  // upward recurrence to nu = mu + N
  double kn = (P.N == 0) ? k0 : k1;
  double km = k0;
  for (int i = 1; i < P.N; ++i) {
    double kp = (2.0 * (mu + double(i)) / x) * kn + km;
    km = kn;
    kn = kp;
  }
  return exp(P.nu * log(x)) * kn;
}

// e^x K_nu(x) for x > 2 by the trapezoidal rule on DLMF 10.32.9.
__device__ __noinline__ double exknu_integral(double x, double nu) {
  const double h = 0.25 / sqrt(x);
  const double hh = 0.5 * h;
  // sinh/cosh of j*h/2 by the addition theorems
  const double sh1 = sinh(hh), ch1 = cosh(hh);
  const double en1 = exp(nu * h);
  double sj = 0.0, cj = 1.0;     // sinh(j h/2), cosh(j h/2) at j = 0
  double ep = 1.0, em = 1.0;     // exp(+-nu j h)
  const double ienu = 1.0 / en1;
  double s = 0.5;
  for (int j = 1; j < 400; ++j) {
    double sn = sj * ch1 + cj * sh1;
    double cn = cj * ch1 + sj * sh1;
    sj = sn;
    cj = cn;
    ep *= en1;
    em *= ienu;
    double term = exp(-2.0 * x * sj * sj) * 0.5 * (ep + em);
    s += term;
    if (term < 1e-17 * s) break;
  }
  return s * h;
}

// C(h) of Eq. (3) without the nugget.
__device__ __forceinline__ double matern_eval(double hdist, const MaternParams& P) {
  double x = hdist * P.inv_ell;
  if (x == 0.0) return P.sigma2;
  if (P.kind != 0) return matern_closed(x, P);
  if (x <= 2.0) return P.norm * xnu_knu_series(x, P);
  double e = exknu_integral(x, P.nu);
  return P.norm * exp(P.nu * log(x) - x) * e;
}

}  // namespace hc
