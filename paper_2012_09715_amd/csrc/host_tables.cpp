// Host FP64 construction of the coefficient tables and the table handle API.
//
// Piecewise constant (Section 2.2, Corollary 2.4): constants on N equal
// intervals, by conditional mean (E), midpoint (C) or inner endpoint (I).
// Dyadic piecewise polynomial (Section 2.3, Theorem 2.5 with r = 1/2, and
// Section 3.3): per-interval L2 projection of Phi^-1 onto polynomials of
// degree d in the local variable s = u 2^(e+1), from the normal equations of
// the proof of Theorem 2.5.  Moments are integrated in z = Phi^-1(u) with
// composite Gauss-Legendre rules; the inverse normal uses Halley steps on
// erfc.  (This code is independent of the test oracle.)
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace aicdf {

static thread_local std::string g_err;

aicdf_status fail(aicdf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

aicdf_status ok() {
  g_err.clear();
  return AICDF_OK;
}

const char* last_error_text() { return g_err.c_str(); }

static const double kInvSqrt2Pi = 0.39894228040143267794;
static const double kSqrt1_2 = 0.70710678118654752440;

double host_Phi(double z) { return 0.5 * std::erfc(-z * kSqrt1_2); }
double host_phi(double z) { return kInvSqrt2Pi * std::exp(-0.5 * z * z); }

// Phi^-1 by Newton steps on log Phi (lower tail) started from the tail
// asymptote, polished by Halley steps on Phi(z) - q; q = min(u, 1-u).
double host_Phi_inv(double u) {
  if (!(u >= 0.0 && u <= 1.0)) return NAN;
  if (u == 0.0) return -INFINITY;
  if (u == 1.0) return INFINITY;
  const bool upper = u > 0.5;
  const double q = upper ? 1.0 - u : u;
  if (q == 0.5) return 0.0;
  // start: z0 solving phi(z)/|z| = q roughly, clipped into the central range
  double z = -std::sqrt(-2.0 * std::log(q));
  if (z > -1.0) z = (q - 0.5) * 2.5066282746310002;
  for (int it = 0; it < 100; ++it) {
    const double f = (q >= 0.25) ? 0.5 * std::erf(z * kSqrt1_2) - (q - 0.5)
                                 : 0.5 * std::erfc(-z * kSqrt1_2) - q;
    const double d = host_phi(z);
    if (d == 0.0) break;
    const double r = f / d;
    const double step = r / (1.0 + 0.5 * z * r);
    z -= step;
    if (std::fabs(step) <= 1e-17 * std::fmax(1.0, std::fabs(z))) break;
  }
  return upper ? -z : z;
}

// n-point Gauss-Legendre nodes/weights on [-1, 1] by Newton on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = -t;
    x[n - 1 - i] = t;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// int_{za}^{zb} f(z) dz with `panels` equal panels of a 24-point rule.
template <class F>
static double integrate_z(F f, double za, double zb, int panels) {
  static std::vector<double> gx, gw;
  static std::once_flag once;
  std::call_once(once, [] { gauss_legendre(24, gx, gw); });
  const double h = (zb - za) / panels;
  double total = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double a = za + p * h, mid = a + 0.5 * h;
    double acc = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) acc += gw[i] * f(mid + 0.5 * h * gx[i]);
    total += 0.5 * h * acc;
  }
  return total;
}

std::vector<double> build_const_table(uint32_t N, int construction) {
  std::vector<double> q(N);
  if (construction == 0) {
    // E(Z | Phi(Z) in I_k) = N (phi(z_k) - phi(z_{k+1})); written as
    // -N phi(z_k) expm1(-(z_{k+1} - z_k)(z_{k+1} + z_k)/2) to avoid cancellation
    // (upper half by antisymmetry).
    std::vector<double> z(N + 1);
    for (uint32_t k = 0; k <= N; ++k) z[k] = host_Phi_inv(double(k) / N);
    for (uint32_t k = 0; k < N / 2; ++k) {
      double v;
      if (k == 0) {
        v = -double(N) * host_phi(z[1]);
      } else {
        const double a = z[k], b = z[k + 1];
        v = -double(N) * host_phi(a) * std::expm1(-0.5 * (b - a) * (b + a));
      }
      q[k] = v;
      q[N - 1 - k] = -v;
    }
  } else if (construction == 1) {
    for (uint32_t k = 0; k < N; ++k) q[k] = host_Phi_inv((k + 0.5) / N);
  } else {
    for (uint32_t k = 0; k < N; ++k) {
      const double lo = double(k) / N, hi = double(k + 1) / N;
      q[k] = host_Phi_inv(lo >= 0.5 ? lo : hi);
    }
  }
  return q;
}

// Small dense solve with partial pivoting (at most 4 x 4).
void solve_small(int n, double* A, double* b) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[p * n + j]);
      std::swap(b[c], b[p]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double acc = b[r];
    for (int j = r + 1; j < n; ++j) acc -= A[r * n + j] * b[j];
    b[r] = acc / A[r * n + r];
  }
}

std::vector<double> build_dyadic_table(uint32_t T, uint32_t degree) {
  const int d1 = int(degree) + 1;
  std::vector<double> tab(size_t(T) * d1, 0.0);
  for (uint32_t e = 1; e < T; ++e) {
    const bool singular = (e == T - 1);
    const double b = std::ldexp(1.0, -int(e));
    const double a = singular ? 0.0 : std::ldexp(1.0, -int(e) - 1);
    const double h = std::ldexp(1.0, -int(e) - 1);
    const double s0 = a / h, s1 = b / h;
    double G[16], m[4];
    for (int i = 0; i < d1; ++i)
      for (int j = 0; j < d1; ++j) {
        const int p = i + j + 1;
        G[i * d1 + j] = (std::pow(s1, p) - std::pow(s0, p)) / p;  // int s^(i+j) ds
      }
    // m_i = int s^i Phi^-1(u) ds = (1/h) int_{za}^{zb} (Phi(z)/h)^i z phi(z) dz
    const double zb = host_Phi_inv(b);
    const double za = singular ? zb - 14.0 : host_Phi_inv(a);
    const int panels = singular ? 112 : 16;
    for (int i = 0; i < d1; ++i) {
      auto f = [&](double z) { return std::pow(host_Phi(z) / h, i) * z * host_phi(z); };
      m[i] = integrate_z(f, za, zb, panels) / h;
    }
    solve_small(d1, G, m);
    for (int j = 0; j < d1; ++j) tab[size_t(e) * d1 + j] = m[j];
  }
  return tab;
}

// Theorem 2.5's bounds for decay rate r: b_0 = 1/2, b_k = b_(k-1) r by FP64
// multiplication, each rounded to FP32 (the thresholds that decide the row).
std::vector<double> geometric_thresholds(double r, uint32_t T) {
  std::vector<double> B(T);
  double b = 0.5;
  for (uint32_t k = 0; k < T; ++k) {
    B[k] = double(float(b));
    b *= r;
  }
  return B;
}

// L2 fits on I_e = [B_e, B_(e-1)) (e < T-1) and the singular (0, B_(T-2)).
// The projection is taken in the Legendre basis of the interval (x = (2u - a
// - b)/(b - a) on [-1, 1]; diagonal Gram matrix (b - a)/(2i + 1)), moments by
// quadrature in z = Phi^-1(u) as for the dyadic rows, and the result is then
// written in powers of s = u / B_e.  The monomial normal equations would lose
// most digits for r near 1, where [1, 1/r) is short.
std::vector<double> build_geometric_table(double r, uint32_t T, uint32_t degree) {
  const int d1 = int(degree) + 1;
  const std::vector<double> B = geometric_thresholds(r, T);
  std::vector<double> tab(size_t(T) * d1, 0.0);
  for (uint32_t e = 1; e < T; ++e) {
    const bool singular = (e == T - 1);
    const double b = B[e - 1], a = singular ? 0.0 : B[e], h = B[e];
    const double w = b - a;
    const double zb = host_Phi_inv(b);
    const double za = singular ? zb - 14.0 : host_Phi_inv(a);
    const int panels = singular ? 112 : 16;
    double leg[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < d1; ++i) {
      auto f = [&](double z) {
        const double x = (2.0 * host_Phi(z) - a - b) / w;
        double p0 = 1.0, p1 = x;  // Bonnet's recurrence for P_i(x)
        for (int k = 1; k < i; ++k) {
          const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
          p0 = p1;
          p1 = p2;
        }
        return (i == 0 ? p0 : p1) * z * host_phi(z);
      };
      leg[i] = (2 * i + 1) / w * integrate_z(f, za, zb, panels);
    }
    // Legendre series -> powers of x (P_2 = (3x^2 - 1)/2, P_3 = (5x^3 - 3x)/2)
    const double px[4] = {leg[0] - 0.5 * leg[2], leg[1] - 1.5 * leg[3], 1.5 * leg[2], 2.5 * leg[3]};
    // powers of x -> powers of s by Horner's rule in the linear map x = alpha s + beta
    const double alpha = 2.0 * h / w, beta = -(a + b) / w;
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = d1 - 1; k >= 0; --k) {
      double nx[4] = {0.0, 0.0, 0.0, 0.0};
      for (int j = 0; j < d1; ++j) {
        nx[j] += beta * cs[j];
        if (j + 1 < d1) nx[j + 1] += alpha * cs[j];
      }
      nx[0] += px[k];
      for (int j = 0; j < d1; ++j) cs[j] = nx[j];
    }
    for (int j = 0; j < d1; ++j) tab[size_t(e) * d1 + j] = cs[j];
  }
  return tab;
}

// Round to nearest even into the given dtype (single rounding from FP64).
static double round_bits(double x, int keep_bits, int min_exp) {
  // keep_bits significant bits; values below 2^min_exp keep the fixed spacing
  // of the subnormal range 2^(min_exp - keep_bits + 1)
  if (x == 0.0 || !std::isfinite(x)) return x;
  int ex;
  std::frexp(x, &ex);  // |x| in [2^(ex-1), 2^ex)
  int lsb = ex - keep_bits;
  if (ex - 1 < min_exp) lsb = min_exp - keep_bits + 1;
  const double scaled = std::ldexp(x, -lsb);  // exact
  return std::ldexp(std::nearbyint(scaled), lsb);  // default mode: nearest even
}

double round_to_dtype(double x, aicdf_dtype t) {
  switch (t) {
    case AICDF_F64: return x;
    case AICDF_F32: return double(float(x));
    case AICDF_F16: return round_bits(x, 11, -14);
    case AICDF_BF16: return round_bits(x, 8, -126);
  }
  return x;
}

}  // namespace aicdf

using namespace aicdf;

extern "C" const char* aicdf_last_error(void) { return last_error_text(); }

static aicdf_status upload_table(aicdf_table* t) {
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  t->device = dev;
  std::vector<float> f32;
  std::vector<double> f64;
  const void* src = nullptr;
  if (t->kind == 0 && t->coef_t == AICDF_F64) {
    f64 = t->host;
    src = f64.data();
    t->dev_bytes = f64.size() * 8;
  } else if (t->kind == 0) {
    f32.assign(t->host.begin(), t->host.end());
    src = f32.data();
    t->dev_bytes = f32.size() * 4;
  } else {
    // 64 rows of four floats (zero padded): one row per lane of a wave;
    // geometric tables append 64 thresholds and 64 scales
    f32.assign(size_t(64) * (t->kind == 2 ? 6 : 4), 0.0f);
    for (uint32_t r = 0; r < t->rows; ++r)
      for (uint32_t c = 0; c < t->cols; ++c) f32[r * 4 + c] = float(t->host[size_t(r) * t->cols + c]);
    if (t->kind == 2) {
      const std::vector<double> B = geometric_thresholds(t->r, t->rows);
      for (uint32_t e = 0; e < t->rows; ++e) {
        f32[256 + e] = float(B[e]);
        f32[320 + e] = float(1.0 / B[e]);
      }
    }
    src = f32.data();
    t->dev_bytes = f32.size() * 4;
  }
  if (hipMalloc(&t->dev, t->dev_bytes) != hipSuccess) {
    t->dev = nullptr;
    return fail(AICDF_ENOMEM, "hipMalloc of %zu bytes for a table failed", t->dev_bytes);
  }
  AICDF_HIP(hipMemcpy(t->dev, src, t->dev_bytes, hipMemcpyHostToDevice));
  return ok();
}

extern "C" aicdf_status aicdf_table_const_create(uint32_t n, int32_t construction,
                                                 aicdf_dtype coef_t, aicdf_table** out) {
  if (!out) return fail(AICDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 2 || n > 65536 || (n & (n - 1)))
    return fail(AICDF_EINVAL, "n_intervals must be a power of two in [2, 65536], got %u", n);
  if (construction < 0 || construction > 2)
    return fail(AICDF_EINVAL, "construction must be 0 (E), 1 (C) or 2 (I)");
  if (!dtype_valid(coef_t)) return fail(AICDF_EDTYPE, "invalid coefficient dtype %d", int(coef_t));
  auto* t = new (std::nothrow) aicdf_table();
  if (!t) return fail(AICDF_ENOMEM, "host allocation failed");
  t->kind = 0;
  t->rows = n;
  t->cols = 1;
  t->construction = construction;
  t->coef_t = coef_t;
  t->dev = nullptr;
  t->host = build_const_table(n, construction);
  for (auto& v : t->host) v = round_to_dtype(v, coef_t);
  aicdf_status st = upload_table(t);
  if (st != AICDF_OK) {
    delete t;
    return st;
  }
  *out = t;
  return ok();
}

extern "C" aicdf_status aicdf_table_const_values(uint32_t n, const double* values, aicdf_dtype coef_t,
                                                 aicdf_table** out) {
  if (!out) return fail(AICDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 2 || n > 65536 || (n & (n - 1)))
    return fail(AICDF_EINVAL, "n_intervals must be a power of two in [2, 65536], got %u", n);
  if (!values) return fail(AICDF_EINVAL, "values is NULL");
  if (!dtype_valid(coef_t)) return fail(AICDF_EDTYPE, "invalid coefficient dtype %d", int(coef_t));
  for (uint32_t k = 0; k < n; ++k)
    if (!std::isfinite(values[k])) return fail(AICDF_EINVAL, "values[%u] is not finite", k);
  auto* t = new (std::nothrow) aicdf_table();
  if (!t) return fail(AICDF_ENOMEM, "host allocation failed");
  t->kind = 0;
  t->rows = n;
  t->cols = 1;
  t->construction = -1;
  t->coef_t = coef_t;
  t->dev = nullptr;
  t->host.assign(values, values + n);
  for (auto& v : t->host) v = round_to_dtype(v, coef_t);
  aicdf_status st = upload_table(t);
  if (st != AICDF_OK) {
    delete t;
    return st;
  }
  *out = t;
  return ok();
}

extern "C" aicdf_status aicdf_table_dyadic_create(uint32_t n_entries, uint32_t degree,
                                                  aicdf_dtype coef_t, aicdf_table** out) {
  if (!out) return fail(AICDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_entries < 3 || n_entries > 64)
    return fail(AICDF_EINVAL, "n_entries must be in [3, 64], got %u", n_entries);
  if (degree > 3) return fail(AICDF_EINVAL, "degree must be in [0, 3], got %u", degree);
  if (coef_t != AICDF_F32 && coef_t != AICDF_F16 && coef_t != AICDF_BF16)
    return fail(AICDF_EDTYPE, "dyadic coefficients must be F32, F16 or BF16");
  auto* t = new (std::nothrow) aicdf_table();
  if (!t) return fail(AICDF_ENOMEM, "host allocation failed");
  t->kind = 1;
  t->rows = n_entries;
  t->cols = degree + 1;
  t->construction = 0;
  t->coef_t = coef_t;
  t->dev = nullptr;
  t->host = build_dyadic_table(n_entries, degree);
  for (auto& v : t->host) v = round_to_dtype(v, coef_t);
  aicdf_status st = upload_table(t);
  if (st != AICDF_OK) {
    delete t;
    return st;
  }
  *out = t;
  return ok();
}

static aicdf_status check_geometric(double r, uint32_t n_entries, uint32_t degree, aicdf_dtype coef_t,
                                    bool allow_f64) {
  if (!(r >= 0.05) || !(r <= 0.95)) return fail(AICDF_EINVAL, "decay rate r must be in [0.05, 0.95]");
  if (n_entries < 3 || n_entries > 64)
    return fail(AICDF_EINVAL, "n_entries must be in [3, 64], got %u", n_entries);
  if (degree > 3) return fail(AICDF_EINVAL, "degree must be in [0, 3], got %u", degree);
  if (coef_t != AICDF_F32 && coef_t != AICDF_F16 && coef_t != AICDF_BF16 && !(allow_f64 && coef_t == AICDF_F64))
    return fail(AICDF_EDTYPE, "geometric coefficients must be F32, F16 or BF16");
  // every threshold a normal FP32 number: the rows stay strictly ordered and
  // their scales 1 / B_e finite
  if (!(geometric_thresholds(r, n_entries).back() >= 0x1p-126))
    return fail(AICDF_EINVAL, "r^(n_entries-1) / 2 underflows FP32 (r = %g, n_entries = %u)", r, n_entries);
  return AICDF_OK;
}

extern "C" aicdf_status aicdf_table_geometric_create(double r, uint32_t n_entries, uint32_t degree,
                                                     aicdf_dtype coef_t, aicdf_table** out) {
  if (!out) return fail(AICDF_EINVAL, "out is NULL");
  *out = nullptr;
  aicdf_status st = check_geometric(r, n_entries, degree, coef_t, false);
  if (st != AICDF_OK) return st;
  auto* t = new (std::nothrow) aicdf_table();
  if (!t) return fail(AICDF_ENOMEM, "host allocation failed");
  t->kind = 2;
  t->rows = n_entries;
  t->cols = degree + 1;
  t->construction = 0;
  t->coef_t = coef_t;
  t->dev = nullptr;
  t->r = r;
  t->host = build_geometric_table(r, n_entries, degree);
  for (auto& v : t->host) v = round_to_dtype(v, coef_t);
  st = upload_table(t);
  if (st != AICDF_OK) {
    delete t;
    return st;
  }
  *out = t;
  return ok();
}

extern "C" aicdf_status aicdf_table_geometric_host(double r, uint32_t n_entries, uint32_t degree, aicdf_dtype coef_t,
                                                   double* host_out, size_t cap) {
  aicdf_status st = check_geometric(r, n_entries, degree, coef_t, true);
  if (st != AICDF_OK) return st;
  if (!host_out) return fail(AICDF_EINVAL, "host_out is NULL");
  const std::vector<double> v = build_geometric_table(r, n_entries, degree);
  if (cap < v.size()) return fail(AICDF_ERANGE, "cap %zu < %zu coefficients", cap, v.size());
  for (size_t i = 0; i < v.size(); ++i) host_out[i] = round_to_dtype(v[i], coef_t);
  return ok();
}

extern "C" aicdf_status aicdf_table_coeffs(const aicdf_table* t, double* host_out, size_t cap,
                                           uint32_t* rows, uint32_t* cols) {
  if (!t) return fail(AICDF_EINVAL, "table is NULL");
  if (rows) *rows = t->rows;
  if (cols) *cols = t->cols;
  if (!host_out) return ok();
  const size_t need = size_t(t->rows) * t->cols;
  if (cap < need) return fail(AICDF_ERANGE, "cap %zu < %zu coefficients", cap, need);
  std::memcpy(host_out, t->host.data(), need * sizeof(double));
  return ok();
}

extern "C" aicdf_status aicdf_table_host_coeffs(int32_t kind, uint32_t n, uint32_t param, aicdf_dtype coef_t,
                                                double* host_out, size_t cap) {
  if (!host_out) return fail(AICDF_EINVAL, "host_out is NULL");
  if (!dtype_valid(coef_t)) return fail(AICDF_EDTYPE, "invalid coefficient dtype");
  std::vector<double> v;
  if (kind == 0) {
    if (n < 2 || n > 65536 || (n & (n - 1))) return fail(AICDF_EINVAL, "n must be a power of two in [2, 65536]");
    if (param > 2) return fail(AICDF_EINVAL, "construction must be 0, 1 or 2");
    v = build_const_table(n, int(param));
  } else if (kind == 1) {
    if (n < 3 || n > 64 || param > 3) return fail(AICDF_EINVAL, "n_entries in [3, 64], degree in [0, 3]");
    v = build_dyadic_table(n, param);
  } else {
    return fail(AICDF_EINVAL, "kind must be 0 (constant) or 1 (dyadic)");
  }
  if (cap < v.size()) return fail(AICDF_ERANGE, "cap %zu < %zu coefficients", cap, v.size());
  for (size_t i = 0; i < v.size(); ++i) host_out[i] = round_to_dtype(v[i], coef_t);
  return ok();
}

extern "C" void aicdf_table_destroy(aicdf_table* t) {
  if (!t) return;
  if (t->dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    (void)hipFree(t->dev);
    (void)hipSetDevice(cur);
  }
  delete t;
}
