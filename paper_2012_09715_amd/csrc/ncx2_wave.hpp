// Wave-cooperative non-central chi-squared CDF / survival function and
// inverse: the 64 lanes of a wavefront evaluate ONE (x, nu, lambda) together.
// Used where a launch has too few independent inverses to fill the GPU (the
// high levels of an MLMC allocation), so that the serial time of one inverse,
// not the throughput, sets the time of the launch.
//
// The sweeps of ncx2_device.hpp are linear recurrences on a two-term state:
//   downward (C):  (D, c)_(j-1) = [[r_j, f_j], [0, f_j]] (D, c)_j,
//                  r_j = j/mu, f_j = r_j (a+j)/y,
//   upward (1-C):  (G, c)_(j+1) = [[r_j, r_j], [0, g_j]] (G, c)_j,
//                  r_j = mu/(j+1), g_j = r_j y/(a+j+1),
// with C = sum D_j (1 - C = sum G_j) and pdf = sum c_j (a+j) / (2y).  A pass
// splits the index range into 64 contiguous chunks, one per lane.  Each lane
// forms the product T of its chunk's matrices and the linear functionals
// that give its chunk's partial sums from the chunk's incoming state; an
// exclusive scan of the T over the lanes (shuffles) gives every lane its
// incoming state from the state at the start of the range, and a butterfly
// reduction sums the partials.  Matrices, states and sums carry a binary
// exponent of their own (all entries are non-negative), so no product
// overflows whatever the range.  Start states, ranges and stopping bounds are
// those of the sequential sweeps, except that a sweep starts further out
// (down to A = 2y for C, up to A = y/2 for 1 - C, at most 4096 terms more),
// where the series (continued fraction) that gives its first term converges
// in a few dozen serial steps; passes continue past the first range while
// the bound on the remaining head (tail) is not met.  The butterfly gives
// every lane the same bits, so the Newton driver around it takes identical
// decisions in all lanes.
#pragma once

#include "ncx2_device.hpp"

namespace aicdf {

// 2^e [[p, r], [0, q]]
struct Ncx2Tri {
  double p, r, q;
  int e;
};

__device__ __forceinline__ void ncx2_norm(Ncx2Tri& t) {
  const double m = fmax(t.p, fmax(t.r, t.q));
  if (m > 0.0) {
    const int k = ilogb(m);
    t.p = ldexp(t.p, -k);
    t.r = ldexp(t.r, -k);
    t.q = ldexp(t.q, -k);
    t.e += k;
  }
}

// Y X (Y applied after X)
__device__ __forceinline__ Ncx2Tri ncx2_compose(const Ncx2Tri& Y, const Ncx2Tri& X) {
  Ncx2Tri z{Y.p * X.p, fma(Y.p, X.r, Y.r * X.q), Y.q * X.q, Y.e + X.e};
  ncx2_norm(z);
  return z;
}

__device__ __forceinline__ Ncx2Tri ncx2_shfl_up(const Ncx2Tri& t, int d) {
  return Ncx2Tri{__shfl_up(t.p, d), __shfl_up(t.r, d), __shfl_up(t.q, d), __shfl_up(t.e, d)};
}

__device__ __forceinline__ Ncx2Tri ncx2_shfl(const Ncx2Tri& t, int src) {
  return Ncx2Tri{__shfl(t.p, src), __shfl(t.r, src), __shfl(t.q, src), __shfl(t.e, src)};
}

// Exclusive scan: lane l receives T_(l-1) ... T_0 (identity in lane 0); `all`
// receives T_63 ... T_0 in every lane.
__device__ __forceinline__ Ncx2Tri ncx2_scan(Ncx2Tri t, int lane, Ncx2Tri& all) {
  for (int d = 1; d < 64; d <<= 1) {
    const Ncx2Tri o = ncx2_shfl_up(t, d);
    if (lane >= d) t = ncx2_compose(t, o);
  }
  all = ncx2_shfl(t, 63);
  Ncx2Tri x = ncx2_shfl_up(t, 1);
  if (lane == 0) x = Ncx2Tri{1.0, 0.0, 1.0, 0};
  return x;
}

// Sum over the wave of m_l 2^(e_l), returned as (mantissa, exponent) in every lane.
__device__ __forceinline__ void ncx2_wave_sum2(double m1, double m2, int e, double& s1, double& s2, int& es) {
  int emax = (m1 > 0.0 || m2 > 0.0) ? e : -100000;
  for (int k = 32; k > 0; k >>= 1) emax = max(emax, __shfl_xor(emax, k));
  double a1 = ldexp(m1, max(e - emax, -2000)), a2 = ldexp(m2, max(e - emax, -2000));
  for (int k = 32; k > 0; k >>= 1) {
    a1 += __shfl_xor(a1, k);
    a2 += __shfl_xor(a2, k);
  }
  s1 = a1;
  s2 = a2;
  es = emax == -100000 ? 0 : emax;
}

// (m, e) += (a, ea)
__device__ __forceinline__ void ncx2_acc(double& m, int& e, double a, int ea) {
  if (!(a > 0.0)) return;
  if (!(m > 0.0)) {
    m = a;
    e = ea;
    return;
  }
  if (ea > e) {
    m = ldexp(m, max(e - ea, -2000)) + a;
    e = ea;
  } else {
    m += ldexp(a, max(ea - e, -2000));
  }
}

constexpr int kNcx2PassTerms = 64 * 16;

// C(x) and pdf(x), the downward sweep shared by the wave.
__device__ inline __noinline__ Ncx2Val ncx2_cdf_wave(double x, double nu, double lam) {
  if (!(x > 0.0)) return Ncx2Val{0.0, 1.0, 0.0};
  if (x > 1.7976931348623157e308) return Ncx2Val{1.0, 0.0, 0.0};
  const int lane = __lane_id();
  const double y = 0.5 * x, a = 0.5 * nu, mu = 0.5 * lam, ly = log(y);
  double jbd, jed;
  ncx2_sweep_range(y, a, mu, jbd, jed);
  // start high enough that the power series for P converges fast (y / A <=
  // 1/2): its terms are serial, the longer sweep is spread over the lanes
  // (je = 0: the single term j = 0)
  if (jed > 0.0) jed = fmax(jed, fmin(ceil(2.0 * y - a), jed + 4096.0));
  const double A = a + jed;
  const double lw = ncx2_logw(jed, mu), lt = ncx2_logt(A, y, ly);
  double P, Q;
  inc_gamma_pq(A, y, 1.0, P, Q);
  const double lc = lw + lt;
  const double lD = (y < A + 1.0) ? lc + log(P) : lw + log(fmax(1.0 - Q * exp(lt), 1e-300));
  const double L = fmax(lD, lc);
  // state at the top of the pass: (D, c) 2^E e^L
  double D = exp(lD - L), c = exp(lc - L);
  int E = 0;
  const double inv_mu = 1.0 / mu, inv_y = 1.0 / y;
  double cdf = 0.0, pa = 0.0;  // totals: (cdf, pa) 2^Et e^L
  int Et = 0;
  int jhi = int(jed), jlo = int(jbd);
  for (int pass = 0; pass < 100000; ++pass) {
    const int n = jhi - jlo + 1;
    const int m = (n + 63) / 64;
    const int my_hi = jhi - lane * m, my_lo = max(jlo, my_hi - m + 1);
    Ncx2Tri T{1.0, 0.0, 1.0, 0};
    double sp = 0.0, sr = 0.0, sq = 0.0;  // sums of T's rows, relative to 2^T.e
    for (int j = my_hi; j >= my_lo; --j) {
      sp += T.p;
      sr += T.r;
      sq = fma(a + j, T.q, sq);
      if (j == 0) break;
      const double rw = j * inv_mu, f = rw * ((a + j) * inv_y);
      T.r = fma(rw, T.r, f * T.q);
      T.p *= rw;
      T.q *= f;
      if (T.p > kNcx2Big || T.r > kNcx2Big || T.q > kNcx2Big) {
        T.p *= kNcx2Small;
        T.r *= kNcx2Small;
        T.q *= kNcx2Small;
        sp *= kNcx2Small;
        sr *= kNcx2Small;
        sq *= kNcx2Small;
        T.e += 600;
      }
    }
    const int es = T.e;
    ncx2_norm(T);
    Ncx2Tri all;
    const Ncx2Tri X = ncx2_scan(T, lane, all);
    // incoming state of this lane's chunk, and its partial sums
    const double Din = fma(X.p, D, X.r * c), cin = X.q * c;
    const double pc = fma(sp, Din, sr * cin), pp = sq * cin;
    double s1, s2;
    int e12;
    ncx2_wave_sum2(pc, pp, es + X.e + E, s1, s2, e12);
    ncx2_acc(cdf, Et, s1, e12);
    ncx2_acc(pa, Et, s2, e12);
    if (jlo == 0) break;
    // state at jlo - 1
    {
      const double Dn = fma(all.p, D, all.r * c), cn = all.q * c;
      const double mx = fmax(Dn, cn);
      const int k = mx > 0.0 ? ilogb(mx) : 0;
      D = ldexp(Dn, -k);
      c = ldexp(cn, -k);
      E += all.e + k;
    }
    const int jn = jlo - 1;
    if (jn < mu && jn < jbd + 1.0) {
      // remaining head below jn: sum w_k P_k <= w_jn r/(1-r); sum c_k <= c_jn rc/(1-rc)
      const double r = jn * inv_mu, rc = r * ((a + jn) * inv_y);
      if (r < 1.0 && rc < 1.0) {
        const double lcdf = log(cdf) + Et * 0.69314718055994531 + L;
        const double log_head = ncx2_logw(double(jn), mu) + log(r / (1.0 - r));
        const double Dr = ldexp(D, E - Et), cr = ldexp(c, E - Et);
        if (log_head <= log(1e-17) + lcdf && Dr <= 1e-17 * cdf && cr * rc / (1.0 - rc) <= 0.5e-17 * pa) {
          cdf += Dr;
          pa = fma(cr, a + jn, pa);
          break;
        }
      }
    }
    jhi = jn;
    jlo = max(0, jn - (kNcx2PassTerms - 1));
  }
  const double e = exp(L + Et * 0.69314718055994531);
  const double C = cdf * e, f = pa * (0.5 * inv_y) * e;
  return Ncx2Val{fmin(C, 1.0), fmax(1.0 - C, 0.0), f};
}

// 1 - C(x) and pdf(x), the upward sweep shared by the wave.
__device__ inline __noinline__ Ncx2Val ncx2_sf_wave(double x, double nu, double lam) {
  if (!(x > 0.0)) return Ncx2Val{0.0, 1.0, 0.0};
  if (x > 1.7976931348623157e308) return Ncx2Val{1.0, 0.0, 0.0};
  const int lane = __lane_id();
  const double y = 0.5 * x, a = 0.5 * nu, mu = 0.5 * lam, ly = log(y);
  double jbd, jed;
  ncx2_sweep_range(y, a, mu, jbd, jed);
  // start low enough that the continued fraction for Q converges fast
  // (A <= y / 2); the longer sweep is spread over the lanes
  if (jed > 0.0) jbd = fmin(jbd, fmax(fmax(0.0, floor(0.5 * y - a)), jbd - 4096.0));
  const double A = a + jbd;
  const double lw = ncx2_logw(jbd, mu), lt = ncx2_logt(A, y, ly);
  double P, Q;
  inc_gamma_pq(A, y, 1.0, P, Q);
  const double lc = lw + lt;
  const double lG = (y < A + 1.0) ? lw + log(fmax(1.0 - P * exp(lt), 1e-300)) : lc + log(Q);
  const double L = fmax(lG, lc);
  double G = exp(lG - L), c = exp(lc - L);
  int E = 0;
  const double muy = mu * y;
  double sf = 0.0, pa = 0.0;
  int Et = 0;
  int jlo = int(jbd), jhi = int(jed);
  for (int pass = 0; pass < 400; ++pass) {
    const int n = jhi - jlo + 1;
    const int m = (n + 63) / 64;
    const int my_lo = jlo + lane * m, my_hi = min(jhi, my_lo + m - 1);
    Ncx2Tri T{1.0, 0.0, 1.0, 0};
    double sp = 0.0, sr = 0.0, sq = 0.0;
    for (int j = my_lo; j <= my_hi; ++j) {
      sp += T.p;
      sr += T.r;
      sq = fma(a + j, T.q, sq);
      const double d = 1.0 / ((j + 1.0) * (a + j + 1.0));
      const double rw = mu * (a + j + 1.0) * d, g = muy * d;
      T.r = rw * (T.r + T.q);
      T.p *= rw;
      T.q *= g;
      if (T.p > kNcx2Big || T.r > kNcx2Big || T.q > kNcx2Big) {
        T.p *= kNcx2Small;
        T.r *= kNcx2Small;
        T.q *= kNcx2Small;
        sp *= kNcx2Small;
        sr *= kNcx2Small;
        sq *= kNcx2Small;
        T.e += 600;
      }
    }
    const int es = T.e;
    ncx2_norm(T);
    Ncx2Tri all;
    const Ncx2Tri X = ncx2_scan(T, lane, all);
    const double Gin = fma(X.p, G, X.r * c), cin = X.q * c;
    const double pc = fma(sp, Gin, sr * cin), pp = sq * cin;
    double s1, s2;
    int e12;
    ncx2_wave_sum2(pc, pp, es + X.e + E, s1, s2, e12);
    ncx2_acc(sf, Et, s1, e12);
    ncx2_acc(pa, Et, s2, e12);
    if (jed == 0.0) break;  // the single term j = 0
    {
      const double Gn = fma(all.p, G, all.r * c), cn = all.q * c;
      const double mx = fmax(Gn, cn);
      const int k = mx > 0.0 ? ilogb(mx) : 0;
      G = ldexp(Gn, -k);
      c = ldexp(cn, -k);
      E += all.e + k;
    }
    const int jn = jhi + 1;
    if (jn > mu && jn > jed - 1.0) {
      // remaining tail from jn: sum w_k Q_k <= w_jn r/(1-r), r = mu/(jn+1)
      const double r = mu / (jn + 1.0), rc = r * (y / (a + jn + 1.0));
      if (rc < 1.0) {
        const double lsf = log(sf) + Et * 0.69314718055994531 + L;
        const double log_tail = ncx2_logw(double(jn), mu) + log(r / (1.0 - r));
        const double Gr = ldexp(G, E - Et), cr = ldexp(c, E - Et);
        if (log_tail <= log(1e-17) + lsf && Gr <= 1e-17 * sf && cr * rc / (1.0 - rc) <= 0.5e-17 * pa) break;
      }
    }
    jlo = jn;
    jhi = jn + kNcx2PassTerms - 1;
  }
  const double e = exp(L + Et * 0.69314718055994531);
  const double S = sf * e, f = pa * (0.5 / y) * e;
  return Ncx2Val{fmax(1.0 - S, 0.0), fmin(S, 1.0), f};
}

struct Ncx2Wave {
  double nu, lam;
  __device__ Ncx2Val cdf(double x) const { return ncx2_cdf_wave(x, nu, lam); }
  __device__ Ncx2Val sf(double x) const { return ncx2_sf_wave(x, nu, lam); }
};

// C_nu^-1(u; lambda) computed by the whole wavefront; every lane must pass
// the same (u, nu, lambda, x0) and receives the same result.  x0 > 0: an
// approximation of the root to start the Newton iteration from.
__device__ inline double ncx2_icdf_wave(double u, double nu, double lam, double x0 = 0.0) {
  if (!(u > 0.0)) return u == 0.0 ? 0.0 : __builtin_nan("");
  if (!(u < 1.0)) return u == 1.0 ? __builtin_inf() : __builtin_nan("");
  const bool upper = u > 0.5;
  return ncx2_solve(upper ? 1.0 - u : u, upper, nu, lam, Ncx2Wave{nu, lam}, nullptr, x0);
}

}  // namespace aicdf
