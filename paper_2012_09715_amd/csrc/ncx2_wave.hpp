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
// exclusive scan of the T over the lanes (register moves between lanes, DPP)
// gives every lane its incoming state from the state at the start of the
// range, and an inclusive scan sums the partials into lane 63.  Matrices, states and sums carry a binary
// exponent of their own (all entries are non-negative), so no product
// overflows whatever the range.  Start states, ranges and stopping bounds are
// those of the sequential sweeps, except that a sweep starts further out
// (down to A = 2y for C, up to A = y/2 for 1 - C, at most 4096 terms more),
// where the series (continued fraction) that gives its first term converges
// in a few dozen serial steps; passes continue past the first range while
// the bound on the remaining head (tail) is not met.  Totals are read back
// from lane 63 as scalars, so every lane holds the same bits and the root
// driver around it takes identical decisions in all lanes.
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

// Cross-lane moves on the vector ALU (DPP), 32 bits at a time: lane l takes
// v from the lane that CTRL names, or keeps `old` where that lane lies outside
// its 16-lane row or the row is masked off (ROWS).  Shift right within rows
// by 1, 2, 4, 8; broadcast of lane 15 of each row to the next row (rows 1
// and 3 written) and of lane 31 to rows 2 and 3; shift of the whole wave
// right by one lane.  They replace LDS-routed shuffles, whose round trips
// set the latency of the one-path-per-wavefront inverse.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

template <int CTRL, int ROWS>
__device__ __forceinline__ int ncx2_dpp(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double ncx2_dpp(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const unsigned lo = unsigned(ncx2_dpp<CTRL, ROWS>(int(o), int(x)));
  const unsigned hi = unsigned(ncx2_dpp<CTRL, ROWS>(int(o >> 32), int(x >> 32)));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ double ncx2_readlane(double v, int l) {
  const long long x = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(x), l));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(x >> 32), l));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// The six steps of an inclusive scan over the 64 lanes with operator
// op(x, y) (x the lane's own value, y the one moved in) and identity `id`:
// four shifts within rows, then the two row broadcasts.
template <class T, class Op>
__device__ __forceinline__ T ncx2_wave_scan(T v, T id, Op op) {
  v = op(v, ncx2_dpp<kDppRowShr1, 0xF>(id, v));
  v = op(v, ncx2_dpp<kDppRowShr2, 0xF>(id, v));
  v = op(v, ncx2_dpp<kDppRowShr4, 0xF>(id, v));
  v = op(v, ncx2_dpp<kDppRowShr8, 0xF>(id, v));
  v = op(v, ncx2_dpp<kDppRowBcast15, 0xA>(id, v));
  v = op(v, ncx2_dpp<kDppRowBcast31, 0xC>(id, v));
  return v;
}

// Sum over the 64 lanes, the same bits in every lane (lane 63's inclusive
// sum, read back as a scalar).
__device__ __forceinline__ double ncx2_wave_total(double v) {
  return ncx2_readlane(ncx2_wave_scan(v, 0.0, [](double x, double y) { return x + y; }), 63);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ Ncx2Tri ncx2_dpp_tri(const Ncx2Tri& t) {
  return Ncx2Tri{ncx2_dpp<CTRL, ROWS>(1.0, t.p), ncx2_dpp<CTRL, ROWS>(0.0, t.r), ncx2_dpp<CTRL, ROWS>(1.0, t.q),
                 ncx2_dpp<CTRL, ROWS>(0, t.e)};
}

// Exclusive scan: lane l receives T_(l-1) ... T_0 (identity in lane 0); `all`
// receives T_63 ... T_0 in every lane.  Composing with the identity leaves a
// normalised matrix unchanged bit for bit, so the lanes that take no value
// in a step need no branch.
__device__ __forceinline__ Ncx2Tri ncx2_scan(Ncx2Tri t, int lane, Ncx2Tri& all) {
  (void)lane;
  t = ncx2_compose(t, ncx2_dpp_tri<kDppRowShr1, 0xF>(t));
  t = ncx2_compose(t, ncx2_dpp_tri<kDppRowShr2, 0xF>(t));
  t = ncx2_compose(t, ncx2_dpp_tri<kDppRowShr4, 0xF>(t));
  t = ncx2_compose(t, ncx2_dpp_tri<kDppRowShr8, 0xF>(t));
  t = ncx2_compose(t, ncx2_dpp_tri<kDppRowBcast15, 0xA>(t));
  t = ncx2_compose(t, ncx2_dpp_tri<kDppRowBcast31, 0xC>(t));
  all = Ncx2Tri{ncx2_readlane(t.p, 63), ncx2_readlane(t.r, 63), ncx2_readlane(t.q, 63),
                __builtin_amdgcn_readlane(t.e, 63)};
  return ncx2_dpp_tri<kDppWaveShr1, 0xF>(t);
}

// Sums over the wave of four values m_i 2^(e_l) with a common per-lane
// exponent, returned as mantissas on one exponent in every lane (the same
// bits in every lane).  m[0..2] >= 0; m[3] may be negative.
__device__ __forceinline__ void ncx2_wave_sum4(const double (&m)[4], int e, double (&s)[4], int& es) {
  const bool any = m[0] > 0.0 || m[1] > 0.0 || m[2] > 0.0 || m[3] != 0.0;
  const int emax = __builtin_amdgcn_readlane(
      ncx2_wave_scan(any ? e : -100000, -100000, [](int x, int y) { return max(x, y); }), 63);
  const int sh = max(e - emax, -2000);
#pragma unroll
  for (int i = 0; i < 4; ++i) s[i] = ncx2_wave_total(ldexp(m[i], sh));
  es = emax == -100000 ? 0 : emax;
}

// m 2^e += a 2^ea for four totals on one exponent.
__device__ __forceinline__ void ncx2_acc4(double (&m)[4], int& e, const double (&a)[4], int ea) {
  if (!(a[0] > 0.0 || a[1] > 0.0 || a[2] > 0.0 || a[3] != 0.0)) return;
  if (!(m[0] > 0.0 || m[1] > 0.0 || m[2] > 0.0 || m[3] != 0.0)) {
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = a[i];
    e = ea;
    return;
  }
  if (ea > e) {
    const int sh = max(e - ea, -2000);
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] = ldexp(m[i], sh) + a[i];
    e = ea;
  } else {
    const int sh = max(ea - e, -2000);
#pragma unroll
    for (int i = 0; i < 4; ++i) m[i] += ldexp(a[i], sh);
  }
}

// S = sum_(k>=0) prod_(i=1..k) y/(A+i), so that P(A, y) = t S with
// t = y^A e^-y / Gamma(A+1) (the power series of the sequential sweeps, for
// y < A + 1), by the wave: lane l takes term k0 + l + 1 of each chunk of 64,
// the terms of a chunk are the prefix products of its ratios (a scan) times
// the product carried in, and a second scan sums them.  The
// ratios fall below 1/2 when A >= 2y, and one chunk then suffices.
__device__ inline double ncx2_series_wave(double A, double y, int lane) {
  double sum = 1.0, carry = 1.0;
  for (int k0 = 0; k0 < 1 << 20; k0 += 64) {
    const double p = ncx2_wave_scan(y / (A + double(k0 + lane + 1)), 1.0, [](double x, double o) { return x * o; });
    const double term = carry * p;
    sum += ncx2_wave_total(term);
    carry = ncx2_readlane(term, 63);
    // the rest is below carry r / (1 - r), r the next ratio (< 1 here)
    const double r = y / (A + double(k0 + 65));
    if (!(r < 1.0) || carry * r <= 1e-17 * sum * (1.0 - r)) break;
  }
  return sum;
}

// log y, log w_j (Poisson weight) and log t_A (as ncx2_logw, ncx2_logt):
// their four logarithms at once, one per lane (lanes 0..3: log y, log mu,
// log (j+1), log (A+1)), and Stirling's series completed on the last two,
// the arithmetic of ncx2_lgamma_stirling bit for bit (the library log-gamma
// where its argument is below 16).
__device__ __forceinline__ void ncx2_logs_wave(double j, double A, double y, double mu, int lane, double& ly,
                                               double& lw, double& lt) {
  const double z = lane == 0 ? y : lane == 1 ? mu : lane == 2 ? j + 1.0 : A + 1.0;
  const double lz = log(z);
  double lg;
  if (!(z >= 16.0)) {
    lg = ncx2_lgamma(z);
  } else {
    const double w = 1.0 / z, w2 = w * w;
    const double s =
        w * (1.0 / 12 + w2 * (-1.0 / 360 + w2 * (1.0 / 1260 + w2 * (-1.0 / 1680 + w2 * (1.0 / 1188 +
                                                                    w2 * (-691.0 / 360360 + w2 * (1.0 / 156)))))));
    lg = (z - 0.5) * lz - z + 0.91893853320467274 + s;
  }
  ly = ncx2_readlane(lz, 0);
  const double lmu = ncx2_readlane(lz, 1), lgj = ncx2_readlane(lg, 2), lgA = ncx2_readlane(lg, 3);
  lw = mu > 0.0 ? -mu + j * lmu - lgj : (j == 0.0 ? 0.0 : -1e308);
  lt = A * ly - y - lgA;
}

constexpr int kNcx2PassTerms = 64 * 16;

// One lane's chunk of the downward sweep: the product T of the step
// matrices of indices j_hi, j_hi - 1, .. (cnt of them) and the sums of its
// rows.  CHECK rescales by 2^-600 when an entry passes 2^600; callers skip it
// when the chunk's growth bound shows that no entry can.
template <bool CHECK>
__device__ __forceinline__ void ncx2_chunk_down(double jd, int cnt, double a, double inv_mu, double inv_y,
                                                Ncx2Tri& T, double& sp, double& sr, double& sq, double& sq2,
                                                double& sq3) {
  // the chunk that ends at j = 0 takes no step below it
  const bool last0 = cnt > 0 && jd - (cnt - 1) == 0.0;
  const int steps = last0 ? cnt - 1 : cnt;
#pragma unroll 2
  for (int i = 0; i < steps; ++i, jd -= 1.0) {
    const double Aj = a + jd;
    sp += T.p;
    sr += T.r;
    sq = fma(Aj, T.q, sq);
    const double qj = Aj * (Aj - 1.0);
    sq2 = fma(qj, T.q, sq2);
    sq3 = fma(qj * T.q, Aj, sq3);
    const double rw = jd * inv_mu, f = rw * (Aj * inv_y);
    T.r = fma(rw, T.r, f * T.q);
    T.p *= rw;
    T.q *= f;
    if (CHECK && (T.p > kNcx2Big || T.r > kNcx2Big || T.q > kNcx2Big)) {
      T.p *= kNcx2Small;
      T.r *= kNcx2Small;
      T.q *= kNcx2Small;
      sp *= kNcx2Small;
      sr *= kNcx2Small;
      sq *= kNcx2Small;
      sq2 *= kNcx2Small;
      sq3 *= kNcx2Small;
      T.e += 600;
    }
  }
  if (last0) {  // the sums of the j = 0 term
    sp += T.p;
    sr += T.r;
    sq = fma(a, T.q, sq);
    const double q0 = a * (a - 1.0);
    sq2 = fma(q0, T.q, sq2);
    sq3 = fma(q0 * T.q, a, sq3);
  }
}

// C(x) and pdf(x), the downward sweep shared by the wave.
__device__ inline __noinline__ Ncx2Val ncx2_cdf_wave(double x, double nu, double lam) {
  if (!(x > 0.0)) return Ncx2Val{0.0, 1.0, 0.0, 0.0};
  if (x > 1.7976931348623157e308) return Ncx2Val{1.0, 0.0, 0.0, 0.0};
  const int lane = __lane_id();
  const double y = 0.5 * x, a = 0.5 * nu, mu = 0.5 * lam;
  double jbd, jed;
  ncx2_sweep_range(y, a, mu, jbd, jed);
  // start high enough that the power series for P converges fast (y / A <=
  // 1/2): its terms are serial, the longer sweep is spread over the lanes
  // (je = 0: the single term j = 0)
  if (jed > 0.0) jed = fmax(jed, fmin(ceil(2.0 * y - a), jed + 4096.0));
  const double A = a + jed;
  double ly, lw, lt;
  ncx2_logs_wave(jed, A, y, mu, lane, ly, lw, lt);
  double P, Q;
  if (y < A + 1.0)
    P = ncx2_series_wave(A, y, lane);
  else
    inc_gamma_pq(A, y, 1.0, P, Q);
  const double lc = lw + lt;
  const double lD = (y < A + 1.0) ? lc + log(P) : lw + log(fmax(1.0 - Q * exp(lt), 1e-300));
  const double L = fmax(lD, lc);
  // state at the top of the pass: (D, c) 2^E e^L
  double D = exp(lD - L), c = exp(lc - L);
  int E = 0;
  const double inv_mu = 1.0 / mu, inv_y = 1.0 / y;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};  // totals (cdf, pa, pb, pq) 2^Et e^L, pa .. pq as in ncx2_cdf
  int Et = 0;
  double wm = 1.0;  // w_(jhi) / w_(jed) = wm 2^we: the scans' products of j/mu
  int we = 0;
  int jhi = int(jed), jlo = int(jbd);
  for (int pass = 0; pass < 100000; ++pass) {
    const int n = jhi - jlo + 1;
    const int m = (n + 63) / 64;
    const int my_hi = jhi - lane * m, my_lo = max(jlo, my_hi - m + 1);
    Ncx2Tri T{1.0, 0.0, 1.0, 0};
    double sp = 0.0, sr = 0.0, sq = 0.0, sq2 = 0.0, sq3 = 0.0;  // sums of T's rows, relative to 2^T.e
    {
      // the step factors j/mu and (j/mu)(a+j)/y grow with j, so every entry
      // grows by at most 2 g per step, g the larger factor at the top index
      const int cnt = my_hi - my_lo + 1;
      const double jt = double(my_hi), g = fmax(jt * inv_mu, jt * inv_mu * ((a + jt) * inv_y));
      if (cnt * (ilogb(fmin(fmax(2.0 * g, 1.0), 0x1p1000)) + 1) < 500)
        ncx2_chunk_down<false>(jt, cnt, a, inv_mu, inv_y, T, sp, sr, sq, sq2, sq3);
      else
        ncx2_chunk_down<true>(jt, cnt, a, inv_mu, inv_y, T, sp, sr, sq, sq2, sq3);
    }
    const int es = T.e;
    ncx2_norm(T);
    Ncx2Tri all;
    const Ncx2Tri X = ncx2_scan(T, lane, all);
    // incoming state of this lane's chunk, and its partial sums
    const double Din = fma(X.p, D, X.r * c), cin = X.q * c;
    const double part[4] = {fma(sp, Din, sr * cin), sq * cin, sq2 * cin, sq3 * cin};
    double sum[4];
    int e12;
    ncx2_wave_sum4(part, es + X.e + E, sum, e12);
    ncx2_acc4(tot, Et, sum, e12);
    if (jlo == 0) break;
    // state at jlo - 1
    {
      wm *= all.p;
      we += all.e;
      const int kw = wm > 0.0 ? ilogb(wm) : 0;
      wm = ldexp(wm, -kw);
      we += kw;
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
        // w_jn r/(1-r) on the scale 2^Et e^L of the totals
        const double head = ncx2_scale(wm * (r / (1.0 - r)), lw - L + (we - Et) * 0.69314718055994531);
        const double Dr = ldexp(D, E - Et), cr = ldexp(c, E - Et);
        if (head <= 1e-17 * tot[0] && Dr <= 1e-17 * tot[0] && cr * rc / (1.0 - rc) <= 0.5e-17 * tot[1]) {
          const double An = a + jn, qn = An * (An - 1.0);
          tot[0] += Dr;
          tot[1] = fma(cr, An, tot[1]);
          tot[2] = fma(cr, qn, tot[2]);
          tot[3] = fma(cr * qn, An, tot[3]);
          break;
        }
      }
    }
    jhi = jn;
    jlo = max(0, jn - (kNcx2PassTerms - 1));
  }
  const double ls = L + Et * 0.69314718055994531;
  const double C = ncx2_scale(tot[0], ls), f = ncx2_scale(tot[1] * (0.5 * inv_y), ls);
  const double fp = ncx2_scale(tot[2] * (0.25 * inv_y * inv_y), ls) - 0.5 * f;
  const double fpp = ncx2_scale((tot[3] - 2.0 * tot[2]) * (0.125 * inv_y * inv_y * inv_y), ls) - fp - 0.25 * f;
  return Ncx2Val{fmin(C, 1.0), fmax(1.0 - C, 0.0), f, fp, fpp};
}

// One lane's chunk of the upward sweep (indices j_lo, j_lo + 1, ..), as
// ncx2_chunk_down.
template <bool CHECK>
__device__ __forceinline__ void ncx2_chunk_up(double jd, int cnt, double a, double mu, double muy, Ncx2Tri& T,
                                              double& sp, double& sr, double& sq, double& sq2, double& sq3) {
#pragma unroll 2
  for (int i = 0; i < cnt; ++i, jd += 1.0) {
    const double Aj = a + jd;
    sp += T.p;
    sr += T.r;
    sq = fma(Aj, T.q, sq);
    const double qj = Aj * (Aj - 1.0);
    sq2 = fma(qj, T.q, sq2);
    sq3 = fma(qj * T.q, Aj, sq3);
    const double d = 1.0 / ((jd + 1.0) * (Aj + 1.0));
    const double rw = mu * (Aj + 1.0) * d, g = muy * d;
    T.r = rw * (T.r + T.q);
    T.p *= rw;
    T.q *= g;
    if (CHECK && (T.p > kNcx2Big || T.r > kNcx2Big || T.q > kNcx2Big)) {
      T.p *= kNcx2Small;
      T.r *= kNcx2Small;
      T.q *= kNcx2Small;
      sp *= kNcx2Small;
      sr *= kNcx2Small;
      sq *= kNcx2Small;
      sq2 *= kNcx2Small;
      sq3 *= kNcx2Small;
      T.e += 600;
    }
  }
}

// 1 - C(x) and pdf(x), the upward sweep shared by the wave.
__device__ inline __noinline__ Ncx2Val ncx2_sf_wave(double x, double nu, double lam) {
  if (!(x > 0.0)) return Ncx2Val{0.0, 1.0, 0.0, 0.0};
  if (x > 1.7976931348623157e308) return Ncx2Val{1.0, 0.0, 0.0, 0.0};
  const int lane = __lane_id();
  const double y = 0.5 * x, a = 0.5 * nu, mu = 0.5 * lam;
  double jbd, jed;
  ncx2_sweep_range(y, a, mu, jbd, jed);
  // start low enough that the continued fraction for Q converges fast
  // (A <= y / 2); the longer sweep is spread over the lanes
  if (jed > 0.0) jbd = fmin(jbd, fmax(fmax(0.0, floor(0.5 * y - a)), jbd - 4096.0));
  const double A = a + jbd;
  double ly, lw, lt;
  ncx2_logs_wave(jbd, A, y, mu, lane, ly, lw, lt);
  double P, Q;
  if (y < A + 1.0)
    P = ncx2_series_wave(A, y, lane);
  else
    inc_gamma_pq(A, y, 1.0, P, Q);
  const double lc = lw + lt;
  const double lG = (y < A + 1.0) ? lw + log(fmax(1.0 - P * exp(lt), 1e-300)) : lc + log(Q);
  const double L = fmax(lG, lc);
  double G = exp(lG - L), c = exp(lc - L);
  int E = 0;
  const double muy = mu * y;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};  // totals (sf, pa, pb, pq) 2^Et e^L
  int Et = 0;
  double wm = 1.0;  // w_(jlo) / w_(jbd) = wm 2^we: the scans' products of mu/(j+1)
  int we = 0;
  int jlo = int(jbd), jhi = int(jed);
  for (int pass = 0; pass < 400; ++pass) {
    const int n = jhi - jlo + 1;
    const int m = (n + 63) / 64;
    const int my_lo = jlo + lane * m, my_hi = min(jhi, my_lo + m - 1);
    Ncx2Tri T{1.0, 0.0, 1.0, 0};
    double sp = 0.0, sr = 0.0, sq = 0.0, sq2 = 0.0, sq3 = 0.0;
    {
      // the step factors mu/(j+1) and mu y/((j+1)(a+j+1)) fall with j: every
      // entry grows by at most 2 g per step, g the larger factor at the bottom
      const int cnt = my_hi - my_lo + 1;
      const double jb = double(my_lo);
      const double g = fmax(mu / (jb + 1.0), muy / ((jb + 1.0) * (a + jb + 1.0)));
      if (cnt * (ilogb(fmin(fmax(2.0 * g, 1.0), 0x1p1000)) + 1) < 500)
        ncx2_chunk_up<false>(jb, cnt, a, mu, muy, T, sp, sr, sq, sq2, sq3);
      else
        ncx2_chunk_up<true>(jb, cnt, a, mu, muy, T, sp, sr, sq, sq2, sq3);
    }
    const int es = T.e;
    ncx2_norm(T);
    Ncx2Tri all;
    const Ncx2Tri X = ncx2_scan(T, lane, all);
    const double Gin = fma(X.p, G, X.r * c), cin = X.q * c;
    const double part[4] = {fma(sp, Gin, sr * cin), sq * cin, sq2 * cin, sq3 * cin};
    double sum[4];
    int e12;
    ncx2_wave_sum4(part, es + X.e + E, sum, e12);
    ncx2_acc4(tot, Et, sum, e12);
    if (jed == 0.0) break;  // the single term j = 0
    {
      wm *= all.p;
      we += all.e;
      const int kw = wm > 0.0 ? ilogb(wm) : 0;
      wm = ldexp(wm, -kw);
      we += kw;
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
        // w_jn r/(1-r) on the scale 2^Et e^L of the totals
        const double tail = ncx2_scale(wm * (r / (1.0 - r)), lw - L + (we - Et) * 0.69314718055994531);
        const double Gr = ldexp(G, E - Et), cr = ldexp(c, E - Et);
        if (tail <= 1e-17 * tot[0] && Gr <= 1e-17 * tot[0] && cr * rc / (1.0 - rc) <= 0.5e-17 * tot[1]) break;
      }
    }
    jlo = jn;
    jhi = jn + kNcx2PassTerms - 1;
  }
  const double ls = L + Et * 0.69314718055994531;
  const double S = ncx2_scale(tot[0], ls), f = ncx2_scale(tot[1] * (0.5 / y), ls);
  const double fp = ncx2_scale(tot[2] * (0.25 / (y * y)), ls) - 0.5 * f;
  const double fpp = ncx2_scale((tot[3] - 2.0 * tot[2]) * (0.125 / (y * y * y)), ls) - fp - 0.25 * f;
  return Ncx2Val{fmax(1.0 - S, 0.0), fmin(S, 1.0), f, fp, fpp};
}

struct Ncx2Wave {
  double nu, lam;
  __device__ Ncx2Val cdf(double x) const { return ncx2_cdf_wave(x, nu, lam); }
  __device__ Ncx2Val sf(double x) const { return ncx2_sf_wave(x, nu, lam); }
};

// C_nu^-1(u; lambda) computed by the whole wavefront; every lane must pass
// the same (u, nu, lambda, x0) and receives the same result.  x0 > 0: an
// approximation of the root to start the iteration from; lga1 as in
// ncx2_solve.
__device__ inline double ncx2_icdf_wave(double u, double nu, double lam, double x0 = 0.0,
                                        double lga1 = __builtin_nan("")) {
  if (!(u > 0.0)) return u == 0.0 ? 0.0 : __builtin_nan("");
  if (!(u < 1.0)) return u == 1.0 ? __builtin_inf() : __builtin_nan("");
  if (!(lam >= 0.0 && lam <= kNcx2MaxLam)) return __builtin_nan("");
  const bool upper = u > 0.5 && (1.0 - u < kNcx2UpperTail || lam > kNcx2UpperLam);
  return ncx2_solve(upper ? 1.0 - u : u, upper, nu, lam, Ncx2Wave{nu, lam}, nullptr, x0, lga1);
}

}  // namespace aicdf
