// Batch exact inverse of the non-central chi-squared CDF (Section 5).  Large
// batches run one inverse per thread (iteration counts differ per lane, the
// divergence the surrogate in the CIR level is meant to avoid); batches too
// small to fill the GPU run one inverse per wavefront with the
// wave-cooperative sweeps, so that the time of a small batch is the serial
// time of one inverse spread over 64 lanes.
#include "internal.hpp"
#include "ncx2_device.hpp"
#include "ncx2_wave.hpp"

using namespace aicdf;

namespace {

// Batches of at most this many inverses run one per wavefront.
constexpr size_t kWaveMaxN = 8192;

// Four waves per SIMD: 128 registers (the compiler's own choice, 130, would
// leave three, 13 % slower over a spread of lambda).
__global__ __launch_bounds__(256, 4) void ncx2_icdf_kernel(double nu, size_t n, const double* __restrict__ u,
                                                        const double* __restrict__ lam, double* __restrict__ x) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    x[i] = ncx2_icdf(u[i], nu, lam[i]);
}

__global__ __launch_bounds__(256) void ncx2_icdf_wave_kernel(double nu, size_t n, const double* __restrict__ u,
                                                             const double* __restrict__ lam,
                                                             double* __restrict__ x) {
  const size_t i = size_t(blockIdx.x) * 4 + threadIdx.x / 64;  // wave-uniform
  if (i >= n) return;
  const double r = ncx2_icdf_wave(u[i], nu, lam[i]);
  if (threadIdx.x % 64 == 0) x[i] = r;
}

}  // namespace

extern "C" aicdf_status ncx2_icdf_exact(double nu, size_t n, const double* u, const double* lambda, double* x,
                                        void* stream) {
  if (!(nu > 0.0) || !(nu < 1e12)) return fail(AICDF_EINVAL, "nu must be in (0, 1e12)");
  if (n == 0) return ok();
  if (!u || !lambda || !x) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * 8, x, n * 8) || overlaps(lambda, n * 8, x, n * 8))
    return fail(AICDF_EALIAS, "x overlaps an input");
  auto s = static_cast<hipStream_t>(stream);
  if (n <= kWaveMaxN) {
    hipLaunchKernelGGL(ncx2_icdf_wave_kernel, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, nu, n, u, lambda, x);
    AICDF_HIP(hipGetLastError());
    return ok();
  }
  int dev = 0, cus = 256;
  AICDF_HIP(hipGetDevice(&dev));
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t need = (n + 255) / 256;
  const size_t maxg = size_t(cus) * 16;
  const unsigned grid = unsigned(need < maxg ? need : maxg);
  hipLaunchKernelGGL(ncx2_icdf_kernel, dim3(grid), dim3(256), 0, s, nu, n, u, lambda, x);
  AICDF_HIP(hipGetLastError());
  return ok();
}
