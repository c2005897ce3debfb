// Matérn covariance of Eq. (3) (Sec. 2.1) on the device:
//   C(h) = sigma^2 / (2^(nu-1) Gamma(nu)) * x^nu * K_nu(x),   x = h / ell,
// with C(0) = sigma^2.  K_nu is evaluated by
//   * the elementary closed forms for nu = 1/2, 3/2, 5/2 (Sec. 2.1 names the
//     nu = 1/2 case the exponential kernel);
//   * Temme's series (N. M. Temme, J. Comput. Phys. 19 (1975) 324-337) for
//     K_mu and K_{mu+1}, |mu| <= 1/2, when x <= 2, followed by the upward
//     recurrence K_{m+1}(x) = (2m/x) K_m(x) + K_{m-1}(x) (DLMF 10.29.1);
//   * for x > 2, Temme's continued fraction CF2 with its normalising sum
//     (Thompson & Barnett 1986) for K_mu, K_{mu+1}, then the same upward
//     recurrence (see exknu_cf2).
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

// x^nu K_nu(x) for 0 < x <= 2 via Temme's series and the (scaled) recurrence.
__device__ __noinline__ double xnu_knu_series(double x, const MaternParams& P) {
  const double mu = P.mu;
  const double lnx2 = -log(0.5 * x);          // ln(2/x)
  const double sig = mu * lnx2;
  const double ep = exp(sig);                 // (x/2)^(-mu)
  const double em = 1.0 / ep;                 // (x/2)^(mu)
  const double coshs = 0.5 * (ep + em);
  // sinh(sig)/sig from sinh itself: (ep - em) / 2 cancels for small sig
  // (1e-13 relative at sig ~ 1e-3)
  const double shs = fabs(sig) < 1e-10 ? 1.0 : sinh(sig) / sig;
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
  // s0 = K_mu, s1 = (x/2) K_{mu+1}.  The upward recurrence runs on the scaled
  // t_m = x^(mu+m) K_(mu+m):  t_(m+1) = 2 (mu + m) t_m + x^2 t_(m-1), so that
  // no large x^(-nu) and small x^nu factors meet at the end
  const double xm = exp(mu * log(x));     // x^mu, |mu| <= 1/2
  double tm = xm * s0;                    // x^mu K_mu
  if (P.N == 0) return tm;
  double tn = 2.0 * xm * s1;              // x^(mu+1) K_(mu+1)
  const double x2 = x * x;
  for (int i = 1; i < P.N; ++i) {
    const double tp = fma(2.0 * (mu + double(i)), tn, x2 * tm);
    tm = tn;
    tn = tp;
  }
  return tn;
}

// e^x K_nu(x) for x > 2 by Temme's continued fraction CF2 (N. M. Temme,
// J. Comput. Phys. 19 (1975); I. J. Thompson and A. R. Barnett, J. Comput.
// Phys. 64 (1986)) for |mu| <= 1/2, then the upward recurrence to nu.
//   K_mu(x) = sqrt(pi) (2x)^mu e^{-x} U(mu + 1/2, 2 mu + 1, 2x)   (DLMF 10.39.10)
// and z_k = U(mu + 1/2 + k, 2 mu + 1, 2x) satisfy (DLMF 13.3.7)
//   z_{k-1} = 2 (x + k) z_k - ((k + 1/2)^2 - mu^2) z_{k+1},
// of which z_k is the minimal solution: a backward recurrence from depth M
// evaluates the continued fraction for z_1 / z_0 (Miller's algorithm), and
// the integral representation of U (DLMF 13.4.4) gives the normalisation
//   sum_k C_k z_k = (2x)^{-mu-1/2},  C_k = (1/2 + mu)_k (1/2 - mu)_k / k!,
// so that e^x K_mu(x) = sqrt(pi / (2x)) / S with S = sum_k C_k z_k / z_0, and
//   K_{mu+1} / K_mu = (mu + x + 1/2 + (mu^2 - 1/4) z_1 / z_0) / x.
// The weights run backwards from C'_M = 1 (C'_{k-1} = C'_k k / ((k - 1/2)^2
// - mu^2)), a common factor that cancels in S.  The depth M = 10 + 150 / x
// keeps the truncation below 2e-16 relative on x > 2 (measured against
// 40-digit values).
__device__ __noinline__ double exknu_cf2(double x, const MaternParams& P) {
  const double mu = P.mu, mu2 = mu * mu;
  double e0, e1;
  if (mu2 == 0.25) {
    // C_k = 0 for k >= 1: S = 1, and the ratio has no z_1 / z_0 term
    e0 = sqrt(M_PI / (2.0 * x));
    e1 = e0 * (mu + x + 0.5) / x;
  } else {
    const int M = 10 + (int)(150.0 / x);
    double zk1 = 0.0, zk = 1.0, w = 1.0, acc = 1.0;   // z_M = 1, C'_M = 1
    for (int k = M; k > 0; --k) {
      const double kh = k + 0.5, km = k - 0.5;
      const double zkm1 = fma(2.0 * (x + k), zk, (mu2 - kh * kh) * zk1);
      w = w * k / (km * km - mu2);
      zk1 = zk;
      zk = zkm1;
      acc = fma(w, zk, acc);
    }
    // acc = sum_k C'_k z_k, and C'_0 = w: S = acc / (w z_0)
    const double S = acc / (w * zk);
    e0 = sqrt(M_PI / (2.0 * x)) / S;
    e1 = e0 * (mu + x + 0.5 + (mu2 - 0.25) * (zk1 / zk)) / x;
  }
  if (P.N == 0) return e0;
  double km = e0, kn = e1;
  for (int i = 1; i < P.N; ++i) {
    const double kp = (2.0 * (mu + double(i)) / x) * kn + km;
    km = kn;
    kn = kp;
  }
  return kn;
}

// C(h) of Eq. (3) without the nugget.
__device__ __forceinline__ double matern_eval(double hdist, const MaternParams& P) {
  double x = hdist * P.inv_ell;
  if (x == 0.0) return P.sigma2;
  if (P.kind != 0) return matern_closed(x, P);
  if (x <= 2.0) return P.norm * xnu_knu_series(x, P);
  // x^nu e^-x (e^x K_nu): the two exponentials separately, so that the
  // rounding of nu log x - x (of order x u) does not enter
  double e = exknu_cf2(x, P);
  return P.norm * exp(P.nu * log(x)) * e * exp(-x);
}

}  // namespace hc
