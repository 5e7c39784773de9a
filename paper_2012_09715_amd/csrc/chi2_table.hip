// The paper's piecewise-polynomial approximation of the non-central
// chi-squared inverse CDF at a fixed nu (Section 5.1): construction on the
// host, the device table, and the streaming transform (u, lambda) -> x~.
//
// Construction.  At knot i (sqrt(y_i) = i/(K-1); y_0 = 0 is the Gaussian
// limit P = Phi^-1(U), y_(K-1) = 1 the central chi-squared, lambda = 0) and
// on each half, every interval's coefficients are the L2 projection of
//   P(t) = (C^-1 - lambda - nu) / (2 sqrt(lambda + nu))
// onto polynomials of degree d in s = t 2^(k+1): the Gram matrix of the
// monomials in s is exact, the moments int s^j P dt use 24-point
// Gauss-Legendre on the regular intervals and on the singular interval
// 16-point rules on the dyadic panels [2^-(m+1), 2^-m], m = n..n+59 (the
// rest of the tail is below FP64 resolution of the moments).  P at a node is
// the exact FP64 inverse of the library (tail-probability form, so that the
// upper half keeps full precision for 1 - U far below 2^-53).  Knots are
// built on host threads.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <thread>

#include "chi2_device.hpp"
#include "internal.hpp"
#include "ncx2_device.hpp"

using namespace aicdf;

struct aicdf_chi2_table {
  double nu;
  uint32_t degree, n_knots, n_int;
  int device;
  std::vector<double> host;  // n_knots x 2 x n_int x (degree + 1), FP64
  f32x4* dev;                // n_knots x 2 x n_int FP32 rows of four
};

namespace {

constexpr uint32_t kMaxKnots = 64, kMaxIntervals = 30;
constexpr int kSingularPanels = 60;

double chi2_P(double t, bool upper, double nu, double y) {
  if (y == 0.0) {
    const double z = host_Phi_inv(t);
    return upper ? -z : z;
  }
  const double lam = nu * (1.0 - y) / y;
  const double s = lam + nu;
  const double x = ncx2_icdf_tail(t, upper, nu, lam);
  return (x - s) / (2.0 * std::sqrt(s));
}

// Coefficients of one half at knot coordinate y: n_int rows of d+1.
void fit_half(double nu, double y, bool upper, uint32_t degree, uint32_t n_int, double* out) {
  static std::vector<double> g24x, g24w, g16x, g16w;
  static std::once_flag once;
  std::call_once(once, [] {
    gauss_legendre(24, g24x, g24w);
    gauss_legendre(16, g16x, g16w);
  });
  const int d1 = int(degree) + 1;
  for (uint32_t k = 1; k <= n_int; ++k) {
    const bool singular = k == n_int;
    const double h = std::ldexp(1.0, -int(k) - 1);
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    auto panel = [&](double a, double b, const std::vector<double>& gx, const std::vector<double>& gw) {
      const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
      for (size_t q = 0; q < gx.size(); ++q) {
        const double t = mid + half * gx[q];
        const double w = half * gw[q] * chi2_P(t, upper, nu, y);
        const double s = t / h;
        double sp = 1.0;
        for (int j = 0; j < d1; ++j, sp *= s) m[j] += w * sp;
      }
    };
    if (!singular) {
      panel(h, 2.0 * h, g24x, g24w);  // [2^-(k+1), 2^-k)
    } else {
      for (int p = 0; p < kSingularPanels; ++p) {
        const double b = std::ldexp(1.0, -int(k) - p), a = 0.5 * b;
        panel(a, b, g16x, g16w);
      }
    }
    // Gram matrix int s^(i+j) dt = h int s^(i+j) ds over s in [s0, s1]
    const double s0 = singular ? 0.0 : 1.0, s1 = 2.0;
    double G[16];
    for (int i = 0; i < d1; ++i)
      for (int j = 0; j < d1; ++j) {
        const int pw = i + j + 1;
        G[i * d1 + j] = h * (std::pow(s1, pw) - std::pow(s0, pw)) / pw;
      }
    solve_small(d1, G, m);
    for (int j = 0; j < d1; ++j) out[size_t(k - 1) * d1 + j] = m[j];
  }
}

aicdf_status check_shape(double nu, uint32_t degree, uint32_t n_knots, uint32_t n_int) {
  if (!(nu > 0.0) || !(nu <= 1e4)) return fail(AICDF_EINVAL, "nu must be in (0, 1e4]");
  if (degree != 1 && degree != 3) return fail(AICDF_EINVAL, "degree must be 1 or 3");
  if (n_knots < 2 || n_knots > kMaxKnots) return fail(AICDF_EINVAL, "n_knots must be in [2, %u]", kMaxKnots);
  if (n_int < 2 || n_int > kMaxIntervals)
    return fail(AICDF_EINVAL, "n_intervals must be in [2, %u]", kMaxIntervals);
  return AICDF_OK;
}

std::vector<double> build(double nu, uint32_t degree, uint32_t n_knots, uint32_t n_int) {
  const size_t half = size_t(n_int) * (degree + 1);
  std::vector<double> tab(size_t(n_knots) * 2 * half);
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const uint32_t jobs = 2 * n_knots;
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < hw; ++w)
    pool.emplace_back([&, w] {
      for (uint32_t j = w; j < jobs; j += hw) {
        const uint32_t knot = j / 2;
        const bool upper = j & 1;
        const double q = double(knot) / (n_knots - 1);
        fit_half(nu, q * q, upper, degree, n_int, tab.data() + size_t(j) * half);
      }
    });
  for (auto& t : pool) t.join();
  return tab;
}

// ---------------------------------------------------------------------------
// Streaming transform: 256-lane work-groups, each thread four float4 of u
// and of lambda (16 samples, 4096 per work-group).  The loads are issued
// first, then the table (a few KB) is staged in LDS, where the per-sample
// gathers of two rows cost far less than through the vector caches (about
// 80% of the HBM peak against 55% for one 64-lane tile per work-group
// reading the table from L1/L2).
constexpr int kBlock = 256;
constexpr int kTiles = 4;
constexpr size_t kPerBlock = size_t(kBlock) * 4 * kTiles;

template <int DEG>
__global__ __launch_bounds__(kBlock) void chi2_transform_kernel(const float* __restrict__ u,
                                                               const float* __restrict__ lam,
                                                               float* __restrict__ x, size_t n, size_t first,
                                                               const f32x4* __restrict__ tab, uint32_t rows,
                                                               Chi2Geom g, int vec_ok) {
  extern __shared__ f32x4 lt[];
  const size_t base = first + size_t(blockIdx.x) * kPerBlock;
  const bool full = vec_ok && base + kPerBlock <= n;  // uniform per work-group
  f32x4 uu[kTiles], ll[kTiles];
  if (full) {
#pragma unroll
    for (int q = 0; q < kTiles; ++q) {
      uu[q] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(u + base) + q * kBlock + threadIdx.x);
      ll[q] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(lam + base) + q * kBlock + threadIdx.x);
    }
  }
  for (uint32_t r = threadIdx.x; r < rows; r += kBlock) lt[r] = tab[r];
  __syncthreads();
  if (full) {
#pragma unroll
    for (int q = 0; q < kTiles; ++q) {
      f32x4 y;
#pragma unroll
      for (int k = 0; k < 4; ++k) y[k] = chi2_approx_x<DEG>(uu[q][k], ll[q][k], lt, g);
      __builtin_nontemporal_store(y, reinterpret_cast<f32x4*>(x + base) + q * kBlock + threadIdx.x);
    }
  } else {
    for (size_t i = base + threadIdx.x; i < n && i < base + kPerBlock; i += kBlock)
      x[i] = chi2_approx_x<DEG>(u[i], lam[i], lt, g);
  }
}

// Sankaran transform: compute-bound (an FP64 exact normal and a power per
// sample), 256-lane work-groups, four samples per thread.
__global__ __launch_bounds__(256) void sankaran_kernel(const float* __restrict__ u, const float* __restrict__ lam,
                                                       float* __restrict__ x, size_t n, float nu, int vec_ok) {
  const size_t i0 = (size_t(blockIdx.x) * 256 + threadIdx.x) * 4;
  if (vec_ok && i0 + 4 <= n) {
    const f32x4 uu = *reinterpret_cast<const f32x4*>(u + i0);
    const f32x4 ll = *reinterpret_cast<const f32x4*>(lam + i0);
    f32x4 y;
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = sankaran_x(uu[k], ll[k], nu);
    *reinterpret_cast<f32x4*>(x + i0) = y;
  } else {
    for (size_t i = i0; i < n && i < i0 + 4; ++i) x[i] = sankaran_x(u[i], lam[i], nu);
  }
}

}  // namespace

namespace aicdf {
Chi2Info chi2_info(const aicdf_chi2_table* t) {
  return Chi2Info{t->nu, t->degree, t->n_knots, t->n_int, t->device, t->dev};
}
}  // namespace aicdf

extern "C" aicdf_status aicdf_chi2_host_coeffs(double nu, uint32_t degree, uint32_t n_knots, uint32_t n_intervals,
                                               double* host_out, size_t cap) {
  aicdf_status st = check_shape(nu, degree, n_knots, n_intervals);
  if (st != AICDF_OK) return st;
  const size_t need = size_t(n_knots) * 2 * n_intervals * (degree + 1);
  if (!host_out || cap < need) return fail(AICDF_EINVAL, "host_out needs %zu doubles", need);
  const std::vector<double> tab = build(nu, degree, n_knots, n_intervals);
  std::copy(tab.begin(), tab.end(), host_out);
  return ok();
}

extern "C" aicdf_status aicdf_chi2_table_create(double nu, uint32_t degree, uint32_t n_knots, uint32_t n_intervals,
                                                aicdf_chi2_table** out) {
  if (!out) return fail(AICDF_EINVAL, "out is NULL");
  *out = nullptr;
  aicdf_status st = check_shape(nu, degree, n_knots, n_intervals);
  if (st != AICDF_OK) return st;
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  auto* t = new aicdf_chi2_table{nu, degree, n_knots, n_intervals, dev, build(nu, degree, n_knots, n_intervals),
                                 nullptr};
  const size_t rows = size_t(n_knots) * 2 * n_intervals;
  std::vector<float> dev_rows(rows * 4, 0.0f);
  for (size_t r = 0; r < rows; ++r)
    for (uint32_t j = 0; j <= degree; ++j) dev_rows[r * 4 + j] = float(t->host[r * (degree + 1) + j]);
  hipError_t e = hipMalloc(&t->dev, rows * sizeof(f32x4));
  if (e == hipSuccess) e = hipMemcpy(t->dev, dev_rows.data(), rows * sizeof(f32x4), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (t->dev) (void)hipFree(t->dev);
    delete t;
    return fail(e == hipErrorOutOfMemory ? AICDF_ENOMEM : AICDF_EHIP, "chi2 table upload: %s",
                hipGetErrorString(e));
  }
  *out = t;
  return ok();
}

extern "C" aicdf_status aicdf_chi2_table_coeffs(const aicdf_chi2_table* t, double* host_out, size_t cap,
                                                size_t* n_written) {
  if (!t) return fail(AICDF_EINVAL, "table is NULL");
  if (n_written) *n_written = t->host.size();
  if (!host_out) return ok();
  if (cap < t->host.size()) return fail(AICDF_EINVAL, "host_out needs %zu doubles", t->host.size());
  std::copy(t->host.begin(), t->host.end(), host_out);
  return ok();
}

extern "C" void aicdf_chi2_table_destroy(aicdf_chi2_table* t) {
  if (!t) return;
  if (t->dev) (void)hipFree(t->dev);
  delete t;
}

extern "C" aicdf_status approx_ncx2_icdf(const aicdf_chi2_table* t, size_t n, const float* u, const float* lambda,
                                         float* x, void* stream) {
  if (!t) return fail(AICDF_EINVAL, "table is NULL");
  if (n == 0) return ok();
  if (!u || !lambda || !x) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * 4, x, n * 4) || overlaps(lambda, n * 4, x, n * 4))
    return fail(AICDF_EALIAS, "x overlaps an input");
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  if (dev != t->device) return fail(AICDF_EINVAL, "table lives on device %d, current device is %d", t->device, dev);
  Chi2Geom g{float(t->nu), float(std::sqrt(t->nu)), float(t->n_knots - 1), t->n_knots - 2, t->n_int};
  const int vec_ok = aligned(u, 16) && aligned(lambda, 16) && aligned(x, 16);
  const uint32_t rows = t->n_knots * 2 * t->n_int;  // <= 64 * 2 * 30 rows = 60 KiB of LDS
  const size_t lds = size_t(rows) * sizeof(f32x4);
  const size_t max_blocks = size_t(1) << 24;
  auto s = static_cast<hipStream_t>(stream);
  for (size_t first = 0; first < n; first += max_blocks * kPerBlock) {
    const size_t blocks = std::min(max_blocks, (n - first + kPerBlock - 1) / kPerBlock);
    if (t->degree == 1)
      hipLaunchKernelGGL(chi2_transform_kernel<1>, dim3(unsigned(blocks)), dim3(kBlock), lds, s, u, lambda, x, n,
                         first, t->dev, rows, g, vec_ok);
    else
      hipLaunchKernelGGL(chi2_transform_kernel<3>, dim3(unsigned(blocks)), dim3(kBlock), lds, s, u, lambda, x, n,
                         first, t->dev, rows, g, vec_ok);
  }
  AICDF_HIP(hipGetLastError());
  return ok();
}

extern "C" aicdf_status approx_ncx2_sankaran(double nu, size_t n, const float* u, const float* lambda, float* x,
                                             void* stream) {
  if (!(nu > 0.0) || !(nu <= 1e4)) return fail(AICDF_EINVAL, "nu must be in (0, 1e4]");
  if (n == 0) return ok();
  if (!u || !lambda || !x) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * 4, x, n * 4) || overlaps(lambda, n * 4, x, n * 4))
    return fail(AICDF_EALIAS, "x overlaps an input");
  const int vec_ok = aligned(u, 16) && aligned(lambda, 16) && aligned(x, 16);
  const size_t per_block = 256 * 4;
  const size_t max_blocks = size_t(1) << 24;
  auto s = static_cast<hipStream_t>(stream);
  for (size_t first = 0; first < n; first += max_blocks * per_block) {
    const size_t m = std::min(n - first, max_blocks * per_block);
    hipLaunchKernelGGL(sankaran_kernel, dim3(unsigned((m + per_block - 1) / per_block)), dim3(256), 0, s, u + first,
                       lambda + first, x + first, m, float(nu), vec_ok);
  }
  AICDF_HIP(hipGetLastError());
  return ok();
}
