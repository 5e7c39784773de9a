// Batch exact inverse of the non-central chi-squared CDF (Section 5), one
// sample per thread.  Iteration counts differ per lane (divergence), which
// is the cost the surrogate in the CIR level is meant to avoid.
#include "internal.hpp"
#include "ncx2_device.hpp"

using namespace aicdf;

namespace {

__global__ __launch_bounds__(256) void ncx2_icdf_kernel(double nu, size_t n, const double* __restrict__ u,
                                                        const double* __restrict__ lam, double* __restrict__ x) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
    x[i] = ncx2_icdf(u[i], nu, lam[i]);
}

}  // namespace

extern "C" aicdf_status ncx2_icdf_exact(double nu, size_t n, const double* u, const double* lambda, double* x,
                                        void* stream) {
  if (!(nu > 0.0) || !(nu < 1e12)) return fail(AICDF_EINVAL, "nu must be in (0, 1e12)");
  if (n == 0) return ok();
  if (!u || !lambda || !x) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * 8, x, n * 8) || overlaps(lambda, n * 8, x, n * 8))
    return fail(AICDF_EALIAS, "x overlaps an input");
  int dev = 0, cus = 256;
  AICDF_HIP(hipGetDevice(&dev));
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t need = (n + 255) / 256;
  const size_t maxg = size_t(cus) * 16;
  const unsigned grid = unsigned(need < maxg ? need : maxg);
  hipLaunchKernelGGL(ncx2_icdf_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), nu, n, u,
                     lambda, x);
  AICDF_HIP(hipGetLastError());
  return ok();
}
