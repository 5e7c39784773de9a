// Exact non-central chi-squared CDF and inverse CDF in FP64 on the device
// (Section 5: the inverse is found by root finding on the CDF, which is the
// Poisson mixture of central chi-squared CDFs, Abramowitz & Stegun 26.4.25).
//
// With y = x/2, a = nu/2, mu = lambda/2, Poisson weights
// w_j = e^-mu mu^j / j! and regularised incomplete gamma functions P, Q:
//   C(x)     = sum_j w_j P(a+j, y)          1 - C(x) = sum_j w_j Q(a+j, y)
//   pdf(x)   = sum_j w_j (1/2) y^(a+j-1) e^-y / Gamma(a+j).
// With t_j = y^(a+j) e^-y / Gamma(a+j+1) and c_j = w_j t_j:
//   P(a+j) = P(a+j+1) + t_j      (additive going down in j)
//   Q(a+j+1) = Q(a+j) + t_j      (additive going up in j)
//   pdf term j = c_j (a+j) / (2y).
// C is therefore summed in ONE downward sweep and 1 - C in ONE upward sweep,
// each using only additions of positive terms (the opposite directions
// subtract and lose all relative accuracy in the far tails).  A sweep starts
// beyond both the peak of c_j ((j+1)(a+j+1) = mu y) and the Poisson peak
// (j = mu), 9 standard deviations plus 16 terms out (the Poisson mass beyond
// is below 1e-17 by the Chernoff bound), from P or Q given by the power
// series (y < a+j+1) or the Lentz continued fraction, and stops once the
// remaining head or tail is below 1e-17 of the sum.  The terms are carried as
// products w_j P_j (or w_j Q_j) and c_j on a running scale (below), so that
// no factor underflows or overflows on the way.  The sweeps divide at most
// once per term (the downward one not at all), and both are kept out of line
// on the device so that the root driver around them stays small in
// registers.
#pragma once

#include "device_common.hpp"

namespace aicdf {

// C, 1 - C, the density f and its first two derivatives in x.  With the
// central densities f_k(x) = (1/2) y^(A-1) e^-y / Gamma(A), A = a+j,
// k = 2A, d f_k/dx = f_k ((A-1)/y - 1)/2 and
// d^2 f_k/dx^2 = f_k ((A-1)(A-2)/y^2 - 2(A-1)/y + 1)/4:
//   f   = sum_j c_j A / (2y),
//   f'  = sum_j c_j A(A-1) / (4y^2) - f/2,
//   f'' = sum_j c_j A(A-1)(A-2) / (8y^3) - f' - f/4.
struct Ncx2Val {
  double cdf, sf, pdf, dpdf, d2pdf = 0.0;
};

// P(A, y) and Q(A, y) with t = y^A e^-y / Gamma(A+1) given (A > 0, y > 0).
__host__ __device__ inline void inc_gamma_pq(double A, double y, double t, double& P, double& Q) {
  if (y < A + 1.0) {
    // P = t * sum_k y^k / ((A+1)...(A+k)), four terms per division: with
    // d1..d4 the next four denominators and r = 1/(d1 d2 d3 d4), the terms
    // are T y/d1 = T y (d2 d3 d4 r), T y^2/(d1 d2) = T y^2 (d3 d4 r), ...
    // (A < 2^60 keeps the product of four denominators far from overflow)
    double term = 1.0, sum = 1.0;
    if (A < 0x1p60) {
      const double y2 = y * y;
      for (int k = 1; k < 100000; k += 4) {
        const double d1 = A + k, d3 = d1 + 2.0, d4 = d1 + 3.0;
        const double d34 = d3 * d4, d234 = (d1 + 1.0) * d34;
        const double r = 1.0 / (d1 * d234);
        const double ty = term * y;
        const double t1 = ty * (d234 * r), t2 = ty * y * (d34 * r), t3 = ty * y2 * (d4 * r);
        term = ty * y2 * y * r;
        sum += t1;
        sum += t2;
        sum += t3;
        sum += term;
        if (term < sum * 1e-17) break;
      }
    } else {
      for (int k = 1; k < 100000; ++k) {
        term *= y / (A + k);
        sum += term;
        if (term < sum * 1e-17) break;
      }
    }
    P = t * sum;
    Q = 1.0 - P;
  } else {
    // Q = t A h, h the continued fraction 1/(y+1-A- 1(1-A)/(y+3-A- ...)) (Lentz)
    const double tiny = 1e-300;
    double b = y + 1.0 - A, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int k = 1; k < 100000; ++k) {
      const double an = -k * (k - A);
      b += 2.0;
      d = an * d + b;
      if (fabs(d) < tiny) d = tiny;
      c = b + an / c;
      if (fabs(c) < tiny) c = tiny;
      d = 1.0 / d;
      const double del = d * c;
      h *= del;
      if (fabs(del - 1.0) < 1e-16) break;
    }
    Q = t * A * h;
    P = 1.0 - Q;
  }
}

// Sweep bounds [jb, je] covering the c_j peak and the Poisson peak.  When
// mu < 1e-40 or mu y < 1e-40 every term beyond j = 0 is below 1e-40 of it
// (D_1/D_0 <= mu, c_1/c_0 = mu y/(a+1), and 1 - C differs from the single
// term by at most C, itself of the size of that term when y is that small),
// and the range is the single term j = 0 (je = 0); this also keeps every
// sweep factor j (a+j)/(mu y) far below the 2^424 that the rescaling by
// 2^-600 can absorb in one step.
__host__ __device__ inline void ncx2_sweep_range(double y, double a, double mu, double& jb, double& je) {
  double js = 0.0;
  if (mu > 0.0) js = fmax(0.0, floor(0.5 * (sqrt(a * a + 4.0 * mu * y) - (a + 2.0)) + 0.5));
  const double lo = fmin(js, mu), hi = fmax(js, mu);
  jb = fmax(0.0, floor(lo - 9.0 * sqrt(lo + 1.0) - 16.0));
  je = ceil(hi + 9.0 * sqrt(hi + 1.0) + 16.0);
  if (!(mu >= 1e-40) || !(mu * y >= 1e-40)) jb = je = 0.0;
}

// m e^ls without underflow or overflow of e^ls alone (the carried sums can
// be far outside the FP64 range of e^ls in the far tails while the product
// is not).
__host__ __device__ inline double ncx2_scale(double m, double ls) {
  if (ls > -700.0 && ls < 700.0) return m * exp(ls);
  if (m == 0.0) return 0.0;
  return copysign(exp(log(fabs(m)) + ls), m);
}

__host__ __device__ inline __noinline__ double ncx2_lgamma(double x) { return lgamma(x); }

// log Gamma(z): for z >= 16 Stirling's series through the z^-13 term (the
// first omitted term is below 3e-20 there), else the library routine.
__host__ __device__ inline double ncx2_lgamma_stirling(double z) {
  if (!(z >= 16.0)) return ncx2_lgamma(z);
  const double w = 1.0 / z, w2 = w * w;
  const double s =
      w * (1.0 / 12 + w2 * (-1.0 / 360 + w2 * (1.0 / 1260 + w2 * (-1.0 / 1680 + w2 * (1.0 / 1188 +
                                                                  w2 * (-691.0 / 360360 + w2 * (1.0 / 156)))))));
  return (z - 0.5) * log(z) - z + 0.91893853320467274 + s;  // 0.918.. = log(2 pi) / 2
}

// log w_j and log t_j.
__host__ __device__ inline double ncx2_logw(double j, double mu) {
  return mu > 0.0 ? -mu + j * log(mu) - ncx2_lgamma_stirling(j + 1.0) : (j == 0.0 ? 0.0 : -1e308);
}
__host__ __device__ inline double ncx2_logt(double A, double y, double ly) {
  return A * ly - y - ncx2_lgamma_stirling(A + 1.0);
}

// The carried terms start at O(1) (scaled by e^-L); whenever one exceeds
// 2^600 every carried value and partial sum is multiplied by 2^-600 and the
// count k of such rescalings grows; the result is sum e^(L + 600 k log 2).  The Poisson weight w_j, needed only for the stopping
// bound, is carried on its own scale e^-Lw.
constexpr double kNcx2Big = 0x1p600;
constexpr double kNcx2Small = 0x1p-600;

// C(x) and pdf(x) by the downward sweep.
__host__ __device__ inline __noinline__ Ncx2Val ncx2_cdf(double x, double nu, double lam) {
  if (!(x > 0.0)) return Ncx2Val{0.0, 1.0, 0.0, 0.0};
  if (x > 1.7976931348623157e308) return Ncx2Val{1.0, 0.0, 0.0, 0.0};
  const double y = 0.5 * x, a = 0.5 * nu, mu = 0.5 * lam, ly = log(y);
  double jb, je;
  ncx2_sweep_range(y, a, mu, jb, je);
  const double A = a + je;
  const double lw = ncx2_logw(je, mu), lt = ncx2_logt(A, y, ly);
  double P, Q;
  inc_gamma_pq(A, y, 1.0, P, Q);  // with t = 1: P holds S = P/t (series) or Q holds A h = Q/t
  const double lc = lw + lt;
  const double lD = (y < A + 1.0) ? lc + log(P) : lw + log(fmax(1.0 - Q * exp(lt), 1e-300));
  const double L = fmax(lD, lc);
  double D = exp(lD - L), c = exp(lc - L), w = 1.0;
  // the stopping bound below, log w + lw - L - 600 k log 2 + log(r/(1-r))
  // <= log(1e-17 C), without logarithms: w r <= T (1 - r) cdf with
  // T = 1e-17 e^(L - lw) 2^(600 k) (0 or inf where that leaves the FP64
  // range: never or always met)
  double T = ncx2_scale(1e-17, L - lw);
  // mu = 0 ends the sweep at j = 0 before inv_mu is used
  const double inv_mu = 1.0 / mu, inv_y = 1.0 / y;
  // pa = sum c_j A_j, pb = sum c_j A_j (A_j - 1), pq = sum c_j A_j^2 (A_j - 1)
  double cdf = 0.0, pa = 0.0, pb = 0.0, pq = 0.0;
  int k = 0;
  // the terms j >= max(jb + 2, 1) cannot end the sweep (the tests below
  // start at j - 1 < jb + 1): without the tests, the same arithmetic
  double dj = je;
  const double jm = fmax(jb + 2.0, 1.0);
  for (; dj >= jm; dj -= 1.0) {
    const double Aj = a + dj;
    cdf += D;
    pa = fma(c, Aj, pa);
    const double qj = Aj * (Aj - 1.0);
    pb = fma(c, qj, pb);
    pq = fma(c * qj, Aj, pq);
    const double rw = dj * inv_mu;
    c = c * rw * (Aj * inv_y);
    w = w * rw;
    D = fma(D, rw, c);
    if (D > kNcx2Big || c > kNcx2Big) {
      D *= kNcx2Small;
      c *= kNcx2Small;
      cdf *= kNcx2Small;
      pa *= kNcx2Small;
      pb *= kNcx2Small;
      pq *= kNcx2Small;
      T *= kNcx2Big;
      ++k;
    }
  }
  for (int j = int(dj);; --j) {
    const double Aj = a + j;
    cdf += D;
    pa = fma(c, Aj, pa);
    const double qj = Aj * (Aj - 1.0);
    pb = fma(c, qj, pb);
    pq = fma(c * qj, Aj, pq);
    if (j == 0) break;
    // step to j - 1: D_(j-1) = (j/mu) D_j + c_(j-1),  c_(j-1) = c_j (j/mu) ((a+j)/y)
    const double rw = j * inv_mu;
    c = c * rw * (Aj * inv_y);
    w = w * rw;
    D = fma(D, rw, c);
    if (D > kNcx2Big || c > kNcx2Big) {
      D *= kNcx2Small;
      c *= kNcx2Small;
      cdf *= kNcx2Small;
      pa *= kNcx2Small;
      pb *= kNcx2Small;
      pq *= kNcx2Small;
      T *= kNcx2Big;
      ++k;
    }
    if (j - 1 < mu && j - 1 < jb + 1.0) {
      // remaining head: sum_(k<j-1) w_k P_k <= w_(j-1) r/(1-r), r = (j-1)/mu;
      // sum of the remaining c_k <= c_(j-1) rc/(1-rc).  Lanes reach this
      // test at different terms, so it is kept to a few multiplications.
      const double r = (j - 1) * inv_mu;
      const double rc = r * ((a + j - 1) * inv_y);
      if (r < 1.0 && rc < 1.0 && w * r <= T * (1.0 - r) * cdf && D <= 1e-17 * cdf &&
          c * rc <= 0.5e-17 * pa * (1.0 - rc)) {
        cdf += D;
        pa = fma(c, a + j - 1, pa);
        const double qj = (a + j - 1) * (a + j - 2);
        pb = fma(c, qj, pb);
        pq = fma(c * qj, a + j - 1, pq);
        break;
      }
    }
  }
  const double ls = L + k * 415.88830833596718;  // e^L 2^(600 k)
  const double C = ncx2_scale(cdf, ls), f = ncx2_scale(pa * (0.5 * inv_y), ls);
  const double fp = ncx2_scale(pb * (0.25 * inv_y * inv_y), ls) - 0.5 * f;
  const double fpp = ncx2_scale((pq - 2.0 * pb) * (0.125 * inv_y * inv_y * inv_y), ls) - fp - 0.25 * f;
  return Ncx2Val{fmin(C, 1.0), fmax(1.0 - C, 0.0), f, fp, fpp};
}

// 1 - C(x) and pdf(x) by the upward sweep.
__host__ __device__ inline __noinline__ Ncx2Val ncx2_sf(double x, double nu, double lam) {
  if (!(x > 0.0)) return Ncx2Val{0.0, 1.0, 0.0, 0.0};
  if (x > 1.7976931348623157e308) return Ncx2Val{1.0, 0.0, 0.0, 0.0};
  const double y = 0.5 * x, a = 0.5 * nu, mu = 0.5 * lam, ly = log(y);
  double jb, je;
  ncx2_sweep_range(y, a, mu, jb, je);
  const double A = a + jb;
  const double lw = ncx2_logw(jb, mu), lt = ncx2_logt(A, y, ly);
  double P, Q;
  inc_gamma_pq(A, y, 1.0, P, Q);
  const double lc = lw + lt;
  const double lG = (y < A + 1.0) ? lw + log(fmax(1.0 - P * exp(lt), 1e-300)) : lc + log(Q);
  const double L = fmax(lG, lc);
  double G = exp(lG - L), c = exp(lc - L), w = 1.0;
  double T = ncx2_scale(1e-17, L - lw);  // the stopping bound's factor, as in ncx2_cdf
  const double muy = mu * y;
  double sf = 0.0, pa = 0.0, pb = 0.0, pq = 0.0;  // as in ncx2_cdf
  int k = 0;
  // the terms j <= je - 2 cannot end the sweep (the test below starts at
  // j + 1 > je - 1; je = 0 is the single term): without the tests, the same
  // arithmetic
  double dj = jb;
  const double jm = je == 0.0 ? -1.0 : fmin(je - 2.0, jb + 399999.0);
  for (; dj <= jm; dj += 1.0) {
    const double Aj = a + dj;
    sf += G;
    pa = fma(c, Aj, pa);
    const double qj = Aj * (Aj - 1.0);
    pb = fma(c, qj, pb);
    pq = fma(c * qj, Aj, pq);
    const double d = 1.0 / ((dj + 1.0) * (Aj + 1.0));
    const double rw = mu * (Aj + 1.0) * d;
    G = rw * (G + c);
    c = c * (muy * d);
    w = w * rw;
    if (G > kNcx2Big || c > kNcx2Big) {
      G *= kNcx2Small;
      c *= kNcx2Small;
      sf *= kNcx2Small;
      pa *= kNcx2Small;
      pb *= kNcx2Small;
      pq *= kNcx2Small;
      T *= kNcx2Big;
      ++k;
    }
  }
  for (int j = int(dj); j < int(jb) + 400000; ++j) {
    const double Aj = a + j;
    sf += G;
    pa = fma(c, Aj, pa);
    const double qj = Aj * (Aj - 1.0);
    pb = fma(c, qj, pb);
    pq = fma(c * qj, Aj, pq);
    if (je == 0.0) break;  // the single term j = 0
    // step to j + 1: G_(j+1) = (mu/(j+1)) (G_j + c_j),  c_(j+1) = c_j (mu/(j+1)) (y/(a+j+1)),
    // with one division: d = 1 / ((j+1)(a+j+1))
    const double d = 1.0 / ((j + 1.0) * (Aj + 1.0));
    const double rw = mu * (Aj + 1.0) * d;
    G = rw * (G + c);
    c = c * (muy * d);
    w = w * rw;
    if (G > kNcx2Big || c > kNcx2Big) {
      G *= kNcx2Small;
      c *= kNcx2Small;
      sf *= kNcx2Small;
      pa *= kNcx2Small;
      pb *= kNcx2Small;
      pq *= kNcx2Small;
      T *= kNcx2Big;
      ++k;
    }
    if (j + 1 > mu && j + 1 > je - 1.0) {
      // remaining tail: sum_(k>j+1) w_k Q_k <= w_(j+1) rw'/(1-rw'), rw' = mu/(j+2)
      // (r < 1 here: j + 2 > mu + 1)
      const double r = mu / (j + 2.0);
      const double rc = r * (y / (Aj + 2.0));
      if (rc < 1.0 && w * r <= T * (1.0 - r) * sf && G <= 1e-17 * sf && c * rc <= 0.5e-17 * pa * (1.0 - rc))
        break;
    }
  }
  const double ls = L + k * 415.88830833596718;  // e^L 2^(600 k)
  const double S = ncx2_scale(sf, ls), f = ncx2_scale(pa * (0.5 / y), ls);
  const double fp = ncx2_scale(pb * (0.25 / (y * y)), ls) - 0.5 * f;
  const double fpp = ncx2_scale((pq - 2.0 * pb) * (0.125 / (y * y * y)), ls) - fp - 0.25 * f;
  return Ncx2Val{fmax(1.0 - S, 0.0), fmin(S, 1.0), f, fp, fpp};
}

// Quick initial value: Patnaik's scaled central chi-squared with the
// Wilson-Hilferty cube-root normal approximation; z from A&S 26.2.23 at the
// tail probability t (lower tail, or upper tail when `upper`).
__host__ __device__ inline __noinline__ double ncx2_guess(double t, bool upper, double nu, double lam) {
  const double tt = sqrt(-2.0 * log(t));
  double z = tt - (2.515517 + tt * (0.802853 + tt * 0.010328)) /
                      (1.0 + tt * (1.432788 + tt * (0.189269 + tt * 0.001308)));
  z = upper ? z : -z;
  const double s = nu + lam, s2 = nu + 2.0 * lam;
  const double rho = s2 / s, k = s * s / s2;
  const double c = 2.0 / (9.0 * k);
  const double b = 1.0 - c + z * sqrt(c);
  return rho * k * b * b * b;
}

// Start for large lambda: Sankaran's approximation (the comparator of
// Section 5.1) in FP64 around the exact normal quantile of the target,
//   c1 = 1 - (2/3)(nu+lambda)(nu+3 lambda)/(nu+2 lambda)^2,
//   c2 = (nu+2 lambda)/(nu+lambda)^2,  c3 = (c1-1)(1-3 c1),
//   B = 1 + c1 c2 (c1 - 1 + (2-c1) c2 c3/2) + c1 sqrt(2 c2)(1 + c2 c3/2) z,
//   x = (nu+lambda) B^(1/c1);
// its relative error falls from ~1e-4 at lambda = 100 to ~1e-6 at 1000
// (against ~3e-4 for the scaled central chi-squared start), which leaves one
// or two root steps.  Returns 0 where B <= 0 (far lower tail).
__host__ __device__ inline __noinline__ double ncx2_sankaran_start(double t, bool upper, double nu, double lam) {
  const double z = upper ? -exact_phi_inv(t) : exact_phi_inv(t);
  const double kl = nu + lam, k2l = nu + 2.0 * lam, k3l = nu + 3.0 * lam;
  const double c1 = 1.0 - (2.0 / 3.0) * kl * k3l / (k2l * k2l);
  const double c2 = k2l / (kl * kl);
  const double c3 = (c1 - 1.0) * (1.0 - 3.0 * c1);
  const double B = 1.0 + c1 * c2 * (c1 - 1.0 + 0.5 * (2.0 - c1) * c2 * c3) +
                   c1 * sqrt(2.0 * c2) * (1.0 + 0.5 * c2 * c3) * z;
  return B > 0.0 ? kl * pow(B, 1.0 / c1) : 0.0;
}

// The step of the highest order that is usable: Householder's third-order
// step g (6 g'^2 - 3 g g'') / (6 g'^3 - 6 g g' g'' + g^2 g'''), else
// Halley's 2 g g' / (2 g'^2 - g g''), else Newton's g / g' (each to be
// subtracted); a higher-order step is usable when it points the way of the
// Newton step and is at most twice as long.  `order` tells which was taken
// (3, 2 or 1).
__host__ __device__ inline double ncx2_step(double g, double dg, double d2g, double d3g, int& order) {
  const double newton = g / dg;
  const double den3 = 6.0 * dg * dg * dg - 6.0 * g * dg * d2g + g * g * d3g;
  if (den3 != 0.0) {
    const double h = g * (6.0 * dg * dg - 3.0 * g * d2g) / den3;
    if (h * newton > 0.0 && fabs(h) <= 2.0 * fabs(newton)) {
      order = 3;
      return h;
    }
  }
  const double den = 2.0 * dg * dg - g * d2g;
  if (den > 0.0) {
    const double h = 2.0 * g * dg / den;
    if (h * newton > 0.0 && fabs(h) <= 2.0 * fabs(newton)) {
      order = 2;
      return h;
    }
  }
  order = 1;
  return newton;
}

// Relative step below which the iteration stops after a step of order 3, 2
// or 1: the error left is of the order of the step's fourth, third or
// second power (1e-16, 1e-15, 1e-18).
__host__ __device__ inline double ncx2_stop(int order) { return order == 3 ? 1e-4 : order == 2 ? 1e-5 : 1e-9; }

// The iteration as an explicit state: ncx2_root_init sets the bracket and
// the start, each evaluation of C (lower form) or 1 - C (upper form) at r.xx
// goes to ncx2_root_update, until r.done; the root is then
// ncx2_root_result(r).
// lga1 = log Gamma(nu/2 + 1).  x0 > 0 inside the bracket replaces the
// built-in initial value (a caller holding an approximation of the root
// passes it here).
struct Ncx2Root {
  double lo, hi, cur;  // bracket and iterate: w = log x (lower form) or x (upper form)
  double xx;           // the point of the next evaluation, e^w or x
  double lt;           // log u (lower form) or log(1 - u) (upper form)
  int it;              // completed iterations
  bool upper, done;
};

__host__ __device__ inline void ncx2_root_init(Ncx2Root& r, double t, bool upper, double nu, double lam, double x0,
                                               double lga1) {
  const double a = 0.5 * nu;
  const double lu = upper ? log1p(-t) : log(t);    // log u
  const double lq = upper ? log(t) : log1p(-t);    // log (1 - u)
  double xlo = 2.0 * exp((lu + lga1) / a);
  double xhi = 2.0 * nu * 0.69314718055994531 + 2.0 * lam - 4.0 * lq;
  if (!(xhi > xlo * 1.001)) xhi = xlo * 1.001 + 1e-300;
  // built-in start: Sankaran's approximation from lambda = 10 on, else (or
  // outside the bracket) the scaled central chi-squared one on the smaller
  // tail probability (from lambda = 10 to 32 Sankaran's start leaves a third
  // evaluation in 2 % of the CIR steps against 30 %)
  double x = x0;
  if (!(x > xlo && x < xhi) && lam >= 10.0) x = ncx2_sankaran_start(t, upper, nu, lam);
  if (!(x > xlo && x < xhi)) x = ncx2_guess(upper || t <= 0.5 ? t : 1.0 - t, upper || t > 0.5, nu, lam);
  if (!(x > xlo && x < xhi)) x = sqrt(xlo) * sqrt(xhi);
  r.upper = upper;
  r.done = false;
  r.it = 0;
  if (!upper) {
    r.lt = lu;
    r.lo = log(xlo);
    r.hi = log(xhi);
    r.cur = log(x);
    r.xx = exp(r.cur);
  } else {
    r.lt = lq;
    r.lo = xlo;
    r.hi = xhi;
    r.cur = x;
    r.xx = x;
  }
}

__host__ __device__ inline double ncx2_root_result(const Ncx2Root& r) { return r.upper ? r.cur : exp(r.cur); }

// One iteration with v = the evaluation at r.xx:
// lower: g(w) = log C(e^w) - log u in w = log x (the lower tail of C is
//        close to a power of x, so g is close to linear in w); with
//        q1 = x f / C, q2 = x^2 f' / C, q3 = x^3 f'' / C:
//        g' = q1,  g'' = q1 + q2 - q1^2,
//        g''' = g'' + 2 q2 + q3 - q1 q2 - 2 q1 g'';
// upper: g(x) = log(1 - u) - log(1 - C(x)) in x (close to linear in x in
//        the upper tail), S = 1 - C:
//        g' = f / S,  g'' = f' / S + g'^2,
//        g''' = f'' / S + (f' / S) g' + 2 g' g''.
// The step is that of ncx2_step.  Steps that leave the bracket are replaced
// by bisection (geometric while the bracket spans more than a factor of
// two).  The iteration stops when a step is below 2e-15 relative, or when a
// step inside the bracket is below ncx2_stop of its order, so the
// confirming evaluation is skipped (measured on the CIR steps: with the
// third-order step the roots stay within 6e-12 of a solve to 2e-15, the
// CDF's own rounding amplified by 2/nu, and take a quarter fewer
// evaluations than with Halley steps); at the latest after 100 iterations.
__host__ __device__ inline void ncx2_root_update(Ncx2Root& r, const Ncx2Val& v) {
  if (!r.upper) {
    const double w = r.cur, xx = r.xx;
    const double g = v.cdf > 0.0 ? log(v.cdf) - r.lt : -1e300;
    if (g == 0.0) {
      r.done = true;
      return;
    }
    if (g < 0.0) r.lo = w; else r.hi = w;
    const double tol = 2e-15 * fmax(1.0, fabs(w));
    double wn = 0.5 * (r.lo + r.hi);
    int order = 0;
    bool good = false;
    if (v.cdf > 0.0 && v.pdf > 0.0) {
      const double q1 = xx * v.pdf / v.cdf, q2 = xx * xx * v.dpdf / v.cdf, q3 = xx * xx * xx * v.d2pdf / v.cdf;
      const double d2g = q1 + q2 - q1 * q1;
      const double d3g = d2g + 2.0 * q2 + q3 - q1 * q2 - 2.0 * q1 * d2g;
      wn = w - ncx2_step(g, q1, d2g, d3g, order);
      good = true;
    }
    if (good && fabs(wn - w) <= tol) {  // converged (may sit on the bracket end)
      r.cur = wn;
      r.done = true;
      return;
    }
    if (!(wn > r.lo && wn < r.hi)) {
      wn = 0.5 * (r.lo + r.hi);
    } else if (good && fabs(wn - w) <= ncx2_stop(order) * fmax(1.0, fabs(w))) {
      r.cur = wn;
      r.done = true;
      return;
    }
    r.cur = wn;
    if (r.hi - r.lo <= tol) {
      r.done = true;
      return;
    }
    r.xx = exp(wn);
  } else {
    const double x = r.cur;
    const double g = v.sf > 0.0 ? r.lt - log(v.sf) : 1e300;
    if (g == 0.0) {
      r.done = true;
      return;
    }
    if (g < 0.0) r.lo = x; else r.hi = x;
    double xn = -1.0;
    int order = 0;
    bool good = false;
    if (v.sf > 0.0 && v.pdf > 0.0) {
      const double dg = v.pdf / v.sf, q2 = v.dpdf / v.sf;
      const double d2g = q2 + dg * dg;
      const double d3g = v.d2pdf / v.sf + q2 * dg + 2.0 * dg * d2g;
      xn = x - ncx2_step(g, dg, d2g, d3g, order);
      good = true;
    }
    if (good && xn > 0.0 && fabs(xn - x) <= 2e-15 * x) {  // converged (may sit on the bracket end)
      r.cur = xn;
      r.done = true;
      return;
    }
    if (!(xn > r.lo && xn < r.hi)) {
      xn = (r.hi > 2.0 * r.lo) ? sqrt(r.lo) * sqrt(r.hi) : 0.5 * (r.lo + r.hi);
    } else if (good && fabs(xn - x) <= ncx2_stop(order) * x) {
      r.cur = xn;
      r.done = true;
      return;
    }
    r.cur = xn;
    if (r.hi - r.lo <= 2e-15 * xn) {
      r.done = true;
      return;
    }
    r.xx = xn;
  }
  if (++r.it >= 100) r.done = true;
}

// Inverse CDF by the iteration above, inside a bracket that is valid before
// any evaluation:
//   lower: C(x) <= P(a, x/2) <= (x/2)^a / Gamma(a+1), so
//          x_lo = 2 (u Gamma(a+1))^(1/a) has C(x_lo) <= u;
//   upper: the Chernoff bound 1 - C(x) <= 2^(nu/2) e^(lambda/2) e^(-x/4)
//          (moment generating function at s = 1/4), so
//          x_hi = 2 nu log 2 + 2 lambda - 4 log(1-u) has 1 - C(x_hi) <= 1-u.
// The target is given as u = t (upper = false) or as the tail probability
// 1 - u = t (upper = true), so that upper-tail targets below the FP64
// spacing near 1 keep full precision; ncx2_icdf takes the upper form only for
// 1 - u < 2^-10 (or lambda > 4096), where 1 - C computed from C would lose
// digits, so that nearly every lane of a batch runs the same (downward) sweep.
// Ev supplies Ncx2Val cdf(x) and Ncx2Val sf(x) for the given (nu, lambda).
// `iters` receives the number of CDF evaluations.
// lga1: log Gamma(nu/2 + 1) when the caller holds it (NaN: computed here).
// The driver is inlined into its callers (the CDF evaluations stay calls):
// called as a function it needs ~200 registers under the calling convention,
// which leaves the one-path-per-thread CIR levels two waves per SIMD instead
// of three.
template <class Ev>
__host__ __device__ __forceinline__ double ncx2_solve(double t, bool upper, double nu, double lam, const Ev& ev,
                                             int* iters, double x0 = 0.0, double lga1 = __builtin_nan("")) {
  Ncx2Root r;
  ncx2_root_init(r, t, upper, nu, lam, x0, lga1 == lga1 ? lga1 : ncx2_lgamma(0.5 * nu + 1.0));
  while (!r.done) ncx2_root_update(r, r.upper ? ev.sf(r.xx) : ev.cdf(r.xx));
  if (iters) *iters = r.it + 1;
  return ncx2_root_result(r);
}

// The sequential evaluator: one lane sums every term.
struct Ncx2Seq {
  double nu, lam;
  __host__ __device__ Ncx2Val cdf(double x) const { return ncx2_cdf(x, nu, lam); }
  __host__ __device__ Ncx2Val sf(double x) const { return ncx2_sf(x, nu, lam); }
};

__host__ __device__ __forceinline__ double ncx2_icdf_tail(double t, bool upper, double nu, double lam,
                                                 int* iters = nullptr, double x0 = 0.0,
                                                 double lga1 = __builtin_nan("")) {
  return ncx2_solve(t, upper, nu, lam, Ncx2Seq{nu, lam}, iters, x0, lga1);
}

// Targets 1 - u below kNcx2UpperTail use the upper-tail form (1 - C by the
// upward sweep), and so does every u > 1/2 when lambda > kNcx2UpperLam: there
// the log-form weights carry exponents of size lambda log lambda, whose
// rounding (relative ~1e-16 of them) is an error of C relative to C, and
// would cost more than 1e-11 of x when only 1 - C is small.  All other
// targets solve C(x) = u with the downward sweep, so that nearly every lane
// of a batch runs the same loop.
constexpr double kNcx2UpperTail = 0x1p-10;
constexpr double kNcx2UpperLam = 4096.0;

// Largest lambda the exact inverse accepts.  The sweeps index their terms
// with int and visit about 18 sqrt(lambda/2) + 32 of them (the upward one at
// most 400000): both stay far within range up to here (127k terms per sweep
// at the bound).  Larger lambda, negative lambda and NaN give NaN.
constexpr double kNcx2MaxLam = 1e8;

// C_nu^-1(u; lambda) for u in [0, 1]: 0 at u = 0, +inf at u = 1, NaN outside
// (and NaN for lambda outside [0, kNcx2MaxLam]).
// x0 > 0: an approximation of the root to start from; lga1 as in ncx2_solve.
__host__ __device__ __forceinline__ double ncx2_icdf(double u, double nu, double lam, int* iters = nullptr,
                                            double x0 = 0.0, double lga1 = __builtin_nan("")) {
  if (!(u > 0.0)) return u == 0.0 ? 0.0 : __builtin_nan("");
  if (!(u < 1.0)) return u == 1.0 ? __builtin_inf() : __builtin_nan("");
  if (!(lam >= 0.0 && lam <= kNcx2MaxLam)) return __builtin_nan("");
  const bool upper = u > 0.5 && (1.0 - u < kNcx2UpperTail || lam > kNcx2UpperLam);
  return ncx2_icdf_tail(upper ? 1.0 - u : u, upper, nu, lam, iters, x0, lga1);
}

}  // namespace aicdf
