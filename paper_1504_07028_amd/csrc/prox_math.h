// Per-pixel closed forms shared by the forward proximity kernel and its
// adjoint: the Schatten-p multiplier of the 2x2 structure tensor and the
// data-term gain, both evaluated in FP64.
#pragma once

#include "segsalsa_internal.h"

namespace segsalsa {

// Multiplier N of the Schatten-p proximity operator for one pixel.
//
// With S = Y^T Y = [[A, B], [B, C]] the structure tensor of the (LK)x2 block
// Y, the proximal point is Y V diag(rho) V^T where sigma_+- = sqrt(eig(S)),
// rho = shrunk(sigma) / sigma (0 where the shrunk value is 0) and V holds the
// eigenvectors of S.  Written as N = alpha I + beta S with beta the divided
// difference (rho_+ - rho_-) / (lambda_+ - lambda_-), expressed in closed
// forms that stay finite and exact as the two eigenvalues merge.
// Prox of tau ||.||_p (1 < p < inf, p != 2) on a pair of singular values
// s1 >= s2 >= 0, written x = (x1, x2).  It is 0 when ||s||_q <= tau (q the dual
// exponent).  Otherwise, with t = x2 / x1 in (0, 1] and
// g(t) = tau (1 + t^p)^{-(p-1)/p} (tau over ||(1, t)||_p^{p-1}), the optimality
// conditions s_i = x_i + tau x_i^{p-1} / ||x||_p^{p-1} give x1 = s1 - g(t),
// x2 = t x1 and the scalar equation
//   F(t) = (s1 - g(t)) t + g(t) t^{p-1} - s2 = 0,   F(0+) = -s2 <= 0 <= F(1) = s1 - s2,
// solved by Newton's method in log t (the power laws are close to linear
// there, also for p near 1) from t = s2 / s1 (the p = 2 direction), kept
// inside the bracket [lo, hi] on t by a geometric bisection.
__device__ inline void lp_shrink2(double s1, double s2, double tau, double p, double& x1, double& x2) {
  x1 = 0.0;
  x2 = 0.0;
  if (!(s1 > 0.0)) return;
  const double q = p / (p - 1.0);
  const double r = s2 / s1;
  if (s1 * pow(1.0 + pow(r, q), 1.0 / q) <= tau) return;
  if (!(s2 > 0.0)) {  // rank one: a scalar soft threshold
    x1 = s1 - tau;
    return;
  }
  const double e = -(p - 1.0) / p;
  double lo = 0.0, hi = 1.0, t = r;
  for (int it = 0; it < 100; ++it) {
    const double tp = pow(t, p), tpm1 = pow(t, p - 1.0);
    const double g = tau * pow(1.0 + tp, e);
    const double F = (s1 - g) * t + g * tpm1 - s2;
    if (F == 0.0) break;
    if (F > 0.0) hi = t;
    else lo = t;
    const double dg = -(p - 1.0) * tpm1 * g / (1.0 + tp);
    const double dFdlogt = t * (s1 - g - dg * t + dg * tpm1) + g * (p - 1.0) * tpm1;
    const double step = F / dFdlogt;
    if (fabs(step) <= 4e-16) {  // converged to rounding: keep the Newton point
      t *= exp(-step);
      break;
    }
    double tn = t * exp(-step);
    if (!(tn > lo && tn < hi)) tn = lo > 0.0 ? sqrt(lo * hi) : 0.5 * hi;
    t = tn;
    if (hi - lo <= 4e-16 * hi) break;
  }
  x1 = s1 - tau * pow(1.0 + pow(t, p), e);
  x2 = t * x1;
}

// GP = false compiles out the general-p branch (its Newton loop would raise
// the register pressure of kernels that never take it).
template <bool GP>
__device__ inline void schatten_multiplier(double A, double B, double C, double tau, int pkind, double pval,
                                           double& n11, double& n12, double& n22) {
  if (!(tau > 0.0)) {  // lambda = 0: prox is the identity
    n11 = 1.0; n12 = 0.0; n22 = 1.0;
    return;
  }
  if (pkind == kSchatten2) {  // Frobenius norm of the block: group shrink
    const double nrm = sqrt(fmax(A + C, 0.0));
    const double rho = nrm > tau ? 1.0 - tau / nrm : 0.0;
    n11 = rho; n12 = 0.0; n22 = rho;
    return;
  }
  const double hs = 0.5 * (A + C);
  const double hd = 0.5 * (A - C);
  const double R = sqrt(hd * hd + B * B);   // (lambda_+ - lambda_-) / 2
  const double lp = hs + R;
  const double lm = fmax(hs - R, 0.0);
  const double sp = sqrt(lp), sm = sqrt(lm);
  if (GP && pkind == kSchattenP) {  // general p: multipliers from the shrunk pair, N = rm I + (rp - rm) e+ e+^T
    double x1, x2;
    lp_shrink2(sp, sm, tau, pval, x1, x2);
    const double rp = sp > 0.0 ? x1 / sp : 0.0;
    const double rmm = sm > 0.0 ? x2 / sm : 0.0;
    const double c2 = R > 0.0 ? hd / R : 1.0, s2 = R > 0.0 ? B / R : 0.0;
    n11 = rmm + (rp - rmm) * 0.5 * (1.0 + c2);
    n22 = rmm + (rp - rmm) * 0.5 * (1.0 - c2);
    n12 = (rp - rmm) * 0.5 * s2;
    return;
  }
  double rm, beta;
  if (pkind == kSchatten1) {  // soft threshold of the singular values
    if (sm > tau) {
      rm = 1.0 - tau / sm;
      beta = tau / (sp * sm * (sp + sm));
    } else if (sp > tau) {
      rm = 0.0;
      beta = (sp - tau) / (sp * 2.0 * R);
    } else {
      n11 = 0.0; n12 = 0.0; n22 = 0.0;
      return;
    }
  } else {  // Schatten-inf: sigma minus its projection on the l1 ball of radius tau
    if (sp + sm <= tau) {
      n11 = 0.0; n12 = 0.0; n22 = 0.0;
      return;
    }
    if (sp - sm >= tau) {
      rm = 1.0;
      beta = -tau / (sp * 2.0 * R);
    } else {
      const double th = 0.5 * (sp + sm - tau);
      rm = th / sm;
      beta = -th / (sp * sm * (sp + sm));
    }
  }
  const double alpha = rm - beta * lm;
  n11 = alpha + beta * A;
  n12 = beta * B;
  n22 = alpha + beta * C;
}

// 1 / (mu t) with t > 0 the root of mu t^2 - mu s t - q = 0 (g1 prox, eq. (10)).
__device__ inline double data_prox_gain(double s, double q, double mu) {
  const double disc = sqrt(s * s + 4.0 * q / mu);
  if (s >= 0.0) return 2.0 / (mu * (s + disc));
  return (disc - s) / (2.0 * q);
}

// Vector-Jacobian product of the Schatten multiplier (the adjoint of the g2
// proximity operator, eq. (13)).  The proximal point is U = Y N(S, tau) with
// S = Y^T Y and N = V diag(g_+, g_-) V^T, g = shrunk(sigma) / sigma a function
// of the two eigenvalues l_+- = sigma_+-^2 of S.  Given the symmetric
// cotangent Nb = sym(Y^T Ubar) of N, it returns
//   Sb = dphi/dS  with phi = <Nb, N(S)>,  as (s11, s12, s22) with
//        <Sb, dS> = s11 dA + 2 s12 dB + s22 dC, so that Y's cotangent gains 2 Y Sb;
//   dtau = <Nb, dN/dtau>.
// In the eigenbasis, the diagonal of Sb is the Jacobian of (g_+, g_-) with
// respect to (l_+, l_-) applied to the diagonal of V^T Nb V, and its
// off-diagonal is the divided difference (g_+ - g_-) / (l_+ - l_-) times
// that of V^T Nb V (the derivative of a spectral function of a symmetric
// matrix).  At merged eigenvalues the divided difference takes its limit and
// V = I serves.
__device__ inline void schatten_multiplier_vjp(double A, double B, double C, double tau, int pkind, double b11,
                                               double b12, double b22, double& s11, double& s12, double& s22,
                                               double& dtau) {
  s11 = 0.0; s12 = 0.0; s22 = 0.0; dtau = 0.0;
  if (pkind == kSchatten2) {  // N = rho I, rho = 1 - tau / sqrt(A + C) above the threshold
    const double nrm = sqrt(fmax(A + C, 0.0));
    if (nrm > tau && nrm > 0.0) {
      const double tr = b11 + b22;
      const double dr = tau > 0.0 ? tau / (2.0 * nrm * nrm * nrm) : 0.0;
      s11 = tr * dr;
      s22 = tr * dr;
      dtau = -tr / nrm;
    }
    return;
  }
  const double hs = 0.5 * (A + C);
  const double hd = 0.5 * (A - C);
  const double R = sqrt(hd * hd + B * B);
  const double lp = hs + R;
  const double lm = fmax(hs - R, 0.0);
  const double sp = sqrt(lp), sm = sqrt(lm);
  const double c2 = R > 0.0 ? hd / R : 1.0;   // cos and sin of twice the eigenvector angle
  const double s2 = R > 0.0 ? B / R : 0.0;
  const double m11 = 0.5 * (b11 + b22) + 0.5 * (b11 - b22) * c2 + b12 * s2;
  const double m22 = 0.5 * (b11 + b22) - 0.5 * (b11 - b22) * c2 - b12 * s2;
  const double m12 = -0.5 * (b11 - b22) * s2 + b12 * c2;
  // dg_a / dl_b, dg_a / dtau and the divided difference
  double gpp = 0.0, gpm = 0.0, gmp = 0.0, gmm = 0.0, gpt = 0.0, gmt = 0.0, beta = 0.0;
  if (!(tau > 0.0)) {  // identity map: no dependence on S, slope in tau from the right
    if (sp > 0.0) gpt = -1.0 / sp;
    if (pkind == kSchatten1 && sm > 0.0) gmt = -1.0 / sm;
    dtau = m11 * gpt + m22 * gmt;
    return;
  }
  if (pkind == kSchatten1) {
    if (sp > tau) {
      gpp = tau / (2.0 * sp * sp * sp);
      gpt = -1.0 / sp;
    }
    if (sm > tau) {
      gmm = tau / (2.0 * sm * sm * sm);
      gmt = -1.0 / sm;
      beta = tau / (sp * sm * (sp + sm));
    } else if (sp > tau) {
      beta = (sp - tau) / (sp * 2.0 * R);
    }
  } else {
    if (sp + sm <= tau) return;  // N = 0 on a neighbourhood
    if (sp - sm >= tau) {        // g_+ = 1 - tau / sigma_+, g_- = 1
      gpp = tau / (2.0 * sp * sp * sp);
      gpt = -1.0 / sp;
      beta = -tau / (sp * 2.0 * R);
    } else {                     // g = th / sigma, th = (sigma_+ + sigma_- - tau) / 2
      const double th = 0.5 * (sp + sm - tau);
      gpp = 0.25 / (sp * sp) - th / (2.0 * sp * sp * sp);
      gmm = 0.25 / (sm * sm) - th / (2.0 * sm * sm * sm);
      gpm = 0.25 / (sp * sm);
      gmp = gpm;
      gpt = -0.5 / sp;
      gmt = -0.5 / sm;
      beta = -th / (sp * sm * (sp + sm));
    }
  }
  const double lbp = m11 * gpp + m22 * gmp;
  const double lbm = m11 * gpm + m22 * gmm;
  const double o = beta * m12;
  s11 = 0.5 * (lbp + lbm) + 0.5 * (lbp - lbm) * c2 - o * s2;
  s22 = 0.5 * (lbp + lbm) - 0.5 * (lbp - lbm) * c2 + o * s2;
  s12 = 0.5 * (lbp - lbm) * s2 + o * c2;
  dtau = m11 * gpt + m22 * gmt;
}

}  // namespace segsalsa
