// Per-stream workspaces, the deterministic final pass over the per-block level
// partials, and the optimal allocation of the nested estimator.
#include <cstdint>
#include <cmath>
#include <map>

#include "mlmc_common.hpp"

namespace aicdf {

namespace {

// One work-group: thread t sums partials t, t+256, ... in order (Neumaier),
// then a fixed-order tree over the 256 values.  The result does not depend on
// scheduling, so repeated calls are bit-identical.  Writes the kSumsOut
// results and clears the fallback counter for the next call on the stream.
__device__ __forceinline__ void reduce_partials_block(const double* __restrict__ partials, unsigned nblocks,
                                                      unsigned long long* __restrict__ counter, double n_paths,
                                                      double* __restrict__ out) {
  __shared__ double red[kSums][kLevelBlock];
  KSum k[kSums];
  // unrolled so that several blocks' loads are in flight together (same order)
#pragma unroll 8
  for (unsigned b = threadIdx.x; b < nblocks; b += kLevelBlock)
#pragma unroll
    for (int j = 0; j < kSums; ++j) k[j].add(partials[size_t(b) * kSums + j]);
#pragma unroll
  for (int j = 0; j < kSums; ++j) red[j][threadIdx.x] = k[j].value();
  __syncthreads();
  for (int o = kLevelBlock / 2; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o)
#pragma unroll
      for (int j = 0; j < kSums; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < kSums) out[threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == kSums) {
    out[kSums] = counter ? double(*counter) : 0.0;
    if (counter) *counter = 0ull;
  }
  if (threadIdx.x == kSums + 1) out[kSums + 1] = n_paths;
}

__global__ __launch_bounds__(kLevelBlock) void reduce_partials_kernel(const double* __restrict__ partials,
                                                                      unsigned nblocks,
                                                                      unsigned long long* __restrict__ counter,
                                                                      double n_paths, double* __restrict__ out) {
  reduce_partials_block(partials, nblocks, counter, n_paths, out);
}

// Work-group j: job j of a batch.
__global__ __launch_bounds__(kLevelBlock) void reduce_batch_kernel(const double* __restrict__ partials, JobSpans sp,
                                                                   unsigned long long* __restrict__ counters,
                                                                   double* __restrict__ out) {
  const uint32_t j = blockIdx.x;
  reduce_partials_block(partials + size_t(sp.start[j]) * kSums, sp.start[j + 1] - sp.start[j],
                        counters ? counters + j : nullptr, sp.n_paths[j], out + size_t(j) * kSumsOut);
}

std::mutex g_ws_mutex;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

}  // namespace

aicdf_status check_level_out(const LevelOut& o) {
  if (!o.host && !o.dev) return fail(AICDF_EINVAL, "the output of the level sums must be non-NULL");
  if (o.dev && (reinterpret_cast<uintptr_t>(o.dev) & 7u))
    return fail(AICDF_EINVAL, "sums_dev must be 8-byte aligned");
  return AICDF_OK;
}

aicdf_status get_workspace(hipStream_t s, Workspace** out) {
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  const auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) {
    *out = it->second;
    return AICDF_OK;
  }
  auto* ws = new (std::nothrow) Workspace();
  if (!ws) return fail(AICDF_ENOMEM, "host allocation failed");
  auto release = [ws]() {
    if (ws->partials) (void)hipFree(ws->partials);
    if (ws->batch_partials) (void)hipFree(ws->batch_partials);
    if (ws->batch_counters) (void)hipFree(ws->batch_counters);
    if (ws->host_result) (void)hipHostFree(ws->host_result);
    if (ws->counter) (void)hipFree(ws->counter);
    if (ws->ev0) (void)hipEventDestroy(ws->ev0);
    if (ws->ev1) (void)hipEventDestroy(ws->ev1);
    delete ws;
  };
  if (hipMalloc(&ws->partials, sizeof(double) * kMaxLevelBlocks * kSums) != hipSuccess ||
      hipHostMalloc(&ws->host_result, sizeof(double) * kSumsOut, hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&ws->counter, sizeof(unsigned long long)) != hipSuccess) {
    release();
    return fail(AICDF_ENOMEM, "allocation of the level workspace failed");
  }
  // the counter starts at zero; every final pass clears it again
  if (hipMemset(ws->counter, 0, sizeof(unsigned long long)) != hipSuccess ||
      hipEventCreate(&ws->ev0) != hipSuccess || hipEventCreate(&ws->ev1) != hipSuccess) {
    release();
    return fail(AICDF_EHIP, "set-up of the level workspace failed");
  }
  g_ws[key] = ws;
  *out = ws;
  return AICDF_OK;
}

aicdf_status get_batch_buffers(Workspace* ws) {
  if (ws->batch_partials) return AICDF_OK;
  double* p = nullptr;
  unsigned long long* c = nullptr;
  if (hipMalloc(&p, sizeof(double) * size_t(kMaxJobs) * kMaxLevelBlocks * kSums) != hipSuccess) {
    return fail(AICDF_ENOMEM, "allocation of the batch partials failed");
  }
  if (hipMalloc(&c, sizeof(unsigned long long) * kMaxJobs) != hipSuccess ||
      hipMemset(c, 0, sizeof(unsigned long long) * kMaxJobs) != hipSuccess) {
    (void)hipFree(p);
    if (c) (void)hipFree(c);
    return fail(AICDF_ENOMEM, "allocation of the batch counters failed");
  }
  ws->batch_partials = p;
  ws->batch_counters = c;
  return AICDF_OK;
}

aicdf_status reduce_batch(const double* partials, const JobSpans& spans, unsigned long long* counters, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(spans.n_jobs), dim3(kLevelBlock), 0, s, partials, spans, counters,
                     out);
  AICDF_HIP(hipGetLastError());
  return ok();
}

aicdf_status begin_level(Workspace* ws, hipStream_t s, const LevelOut& o) {
  if (o.host) AICDF_HIP(hipEventRecord(ws->ev0, s));
  return AICDF_OK;
}

aicdf_status finish_level(Workspace* ws, unsigned nblocks, hipStream_t s, double n_paths, const LevelOut& o) {
  // the host path's final pass writes straight into pinned host memory: no
  // copy is queued, and the wait for the stream makes its writes visible
  double* dst = o.host ? ws->host_result : o.dev;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kLevelBlock), 0, s, ws->partials, nblocks, ws->counter,
                     n_paths, dst);
  AICDF_HIP(hipGetLastError());
  if (!o.host) return ok();
  AICDF_HIP(hipEventRecord(ws->ev1, s));
  AICDF_HIP(hipStreamSynchronize(s));
  double res[kSumsOut];
  for (int j = 0; j < kSumsOut; ++j) res[j] = ws->host_result[j];
  float ms = 0.0f;
  AICDF_HIP(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
  aicdf_level_sums* out = o.host;
  out->n = n_paths;
  for (int j = 0; j < 4; ++j) out->sum[j] = res[j];
  out->sum_pf = res[4];
  out->sum_pc = res[5];
  out->kernel_ms = ms;
  out->fallbacks = static_cast<uint64_t>(res[kSums]);
  out->reserved = 0;
  return ok();
}

aicdf_status empty_level(hipStream_t s, const LevelOut& o) {
  if (o.host) {
    *o.host = aicdf_level_sums{};
    return ok();
  }
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kLevelBlock), 0, s, nullptr, 0u, nullptr, 0.0, o.dev);
  AICDF_HIP(hipGetLastError());
  return ok();
}

aicdf_status reduce_partials_to(const double* partials, unsigned nblocks, double n_paths, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kLevelBlock), 0, s, partials, nblocks, nullptr, n_paths,
                     out);
  AICDF_HIP(hipGetLastError());
  return ok();
}

}  // namespace aicdf

using namespace aicdf;

extern "C" aicdf_status mlmc_allocate(uint32_t L, double eps, const double* vh, const double* ch, const double* v2,
                                      const double* c2, const double* v4, const double* c4, double* mh, double* m2,
                                      double* m4, double* T_hat, double* T_tilde) {
  if (L == 0 || !(eps > 0.0)) return fail(AICDF_EINVAL, "need n_levels > 0 and eps > 0");
  if (!vh || !ch || !v2 || !c2 || !v4 || !c4 || !T_hat || !T_tilde) return fail(AICDF_EINVAL, "NULL array");
  double sh = 0.0, st = 0.0;
  for (uint32_t l = 0; l < L; ++l) {
    if (!(vh[l] >= 0.0 && v2[l] >= 0.0 && v4[l] >= 0.0) || !(ch[l] > 0.0 && c2[l] > 0.0 && c4[l] > 0.0))
      return fail(AICDF_EINVAL, "level %u: variances must be >= 0 and costs > 0", l);
    sh += std::sqrt(vh[l] * ch[l]);
    st += std::sqrt(v2[l] * c2[l]) + std::sqrt(v4[l] * c4[l]);
  }
  const double Th = 2.0 / (eps * eps) * sh * sh;
  const double Tt = 2.0 / (eps * eps) * st * st;
  for (uint32_t l = 0; l < L; ++l) {
    if (mh) mh[l] = std::sqrt(2.0 * Th * vh[l] / ch[l]) / eps;
    if (m2) m2[l] = std::sqrt(2.0 * Tt * v2[l] / c2[l]) / eps;
    if (m4) m4[l] = std::sqrt(2.0 * Tt * v4[l] / c4[l]) / eps;
  }
  *T_hat = Th;
  *T_tilde = Tt;
  return ok();
}
