// Shared pieces of the fused MLMC level kernels: FP64 level sums (per-thread
// sums, block tree reduction into per-block partials, one deterministic
// Neumaier pass over the partials), approximate-normal tables staged in LDS,
// and the library's per-stream workspaces.
#pragma once

#include <mutex>

#include "device_common.hpp"
#include "internal.hpp"

namespace aicdf {

constexpr int kSums = 6;  // Y, Y^2, Y^3, Y^4, P_f, P_c
constexpr int kLevelBlock = 256;
constexpr int kMaxLevelBlocks = 4096;

// Neumaier compensated sum.
struct KSum {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

// Per-thread sums of one level in plain FP64: a thread adds n_paths / 2^20
// paths (about a hundred at 10^8 paths), so the rounding stays near
// n eps of the absolute sum, far below the statistical error of the level;
// the block tree and the final Neumaier pass over the blocks' partials carry
// the rest.
struct LevelAcc {
  double k[kSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  __device__ __forceinline__ void add(double y, double pf, double pc) {
    const double y2 = y * y;
    k[0] += y;
    k[1] += y2;
    k[2] = fma(y2, y, k[2]);
    k[3] = fma(y2, y2, k[3]);
    k[4] += pf;
    k[5] += pc;
  }
};

// Block-wide tree reduction of the per-thread sums into partials[bid].
__device__ __forceinline__ void block_reduce_store(const LevelAcc& acc, double* __restrict__ partials,
                                                   uint32_t bid) {
  __shared__ double red[kSums][kLevelBlock];
#pragma unroll
  for (int j = 0; j < kSums; ++j) red[j][threadIdx.x] = acc.k[j];
  __syncthreads();
  for (int o = kLevelBlock / 2; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) {
#pragma unroll
      for (int j = 0; j < kSums; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x < kSums) partials[size_t(bid) * kSums + threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ void block_reduce_store(const LevelAcc& acc, double* __restrict__ partials) {
  block_reduce_store(acc, partials, blockIdx.x);
}

// Level-batched calls (one launch for many (level, kind) jobs of one
// estimator): at most kMaxJobs jobs; job j owns the work-groups
// [start[j], start[j+1]) of the launch, as many as its own level call would
// launch, and its partials sit at the same offsets of the batch's partials.
constexpr int kMaxJobs = 24;

struct JobSpans {
  uint32_t start[kMaxJobs + 1];
  double n_paths[kMaxJobs];
  uint32_t n_jobs;
};

// The final pass of a batch: one work-group per job, each the single-call
// final pass over its own partials (the same summation order, so each job's
// sums are bit-identical to its level call's); out: n_jobs x kSumsOut.
// counters: one fallback counter per job (or NULL), read and cleared.
aicdf_status reduce_batch(const double* partials, const JobSpans& spans, unsigned long long* counters, double* out,
                          hipStream_t s);

// Host side: one workspace per (device, stream) a level call has used
// (created on first use, kept until the process ends), so that calls on
// different streams can run concurrently.  A synchronous call holds its
// workspace's mutex from the first launch to the copy-out, which serialises
// calls that share a stream; a stream-ordered call holds it while it enqueues,
// and the stream's order keeps its partials and counter apart from those of
// the next call on that stream.  The fallback counter is zero between calls:
// zeroed at creation, read and cleared by the final pass of each call.
struct Workspace {
  double* partials = nullptr;  // kMaxLevelBlocks * kSums doubles
  double* batch_partials = nullptr;            // kMaxJobs * kMaxLevelBlocks * kSums doubles (first batch call)
  unsigned long long* batch_counters = nullptr;  // kMaxJobs fallback counters, zero between calls
  double* host_result = nullptr;  // kSumsOut doubles of pinned host memory, written by the final pass
  unsigned long long* counter = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::mutex mu;
};

// Layout of a level's results in device memory: the kSums sums, then the
// fallback count and the number of paths (both exact in FP64).
constexpr int kSumsOut = 8;

// Where a level call delivers its sums: to the host (synchronous call, with
// the level kernel's device time) or to caller-owned device memory (stream
// ordered, no wait, no timing).
struct LevelOut {
  aicdf_level_sums* host = nullptr;
  double* dev = nullptr;
};

aicdf_status check_level_out(const LevelOut& o);

aicdf_status get_workspace(hipStream_t s, Workspace** ws);

// The workspace's batch buffers, allocated on its first batched call.
aicdf_status get_batch_buffers(Workspace* ws);

// Records the start event of a synchronous call (no-op for a stream-ordered one).
aicdf_status begin_level(Workspace* ws, hipStream_t s, const LevelOut& o);

// The final pass over the level kernel's nblocks partials; a synchronous call
// then waits and fills o.host.
aicdf_status finish_level(Workspace* ws, unsigned nblocks, hipStream_t s, double n_paths, const LevelOut& o);

// A call of zero paths: all-zero results (enqueued for a stream-ordered call).
aicdf_status empty_level(hipStream_t s, const LevelOut& o);

// The final pass over nblocks partials at `partials` (device memory the
// caller provides), writing the kSumsOut results to `out` (device memory) in
// stream order; no fallback counter (reported as 0).  Allocates nothing.
aicdf_status reduce_partials_to(const double* partials, unsigned nblocks, double n_paths, double* out,
                                hipStream_t s);

}  // namespace aicdf
