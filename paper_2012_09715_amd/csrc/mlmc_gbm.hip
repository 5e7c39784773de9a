// Fused MLMC level of geometric Brownian motion (Section 4): counter-based
// uniforms -> exact and/or approximate normals -> coupled fine (2^l steps)
// and coarse (2^(l-1) steps, pairwise-summed Wiener increments) paths ->
// payoff -> compensated FP64 level sums.  One path per thread and iteration
// of a grid-stride loop; the path state lives in registers; the
// approximation's table is staged once per work-group in LDS.
//
// The correction kind carries the approximate path X~ and the difference
// e = X^ - X~ instead of two full paths, so that the four-way difference
// D = (P^_f - P^_c) - (P~_f - P~_c) is formed without cancellation:
//   X~' = X~ g(dW~),   e' = e g(dW^) + X~ (g(dW^) - g(dW~)),
// with g(dW) = 1 + r h + sigma dW (+ sigma^2 (dW^2 - h)/2 for Milstein) and
// g(dW^) - g(dW~) = sigma d (+ sigma^2 d (dW^ + dW~)/2), d = dW^ - dW~ taken
// from the FP64 exact normal minus the FP32 approximate one.
//
// Calls with few paths of many steps (the high levels of an MLMC allocation,
// whose time is the serial time of one path) run one path per group of
// G = min(64, 2^l / 2) lanes instead: every scheme step maps the state
// linearly,
//   X' = g X  (EXACT, APPROX),   (X~, e)' = [[g~, 0], [dg, g^]] (X~, e),
// so each lane forms the product of the step maps of its 2^l/G consecutive
// steps (draws and normals included) and an ordered tree of shuffles
// multiplies the G lane products; the group's first lane applies the result
// to (S0, 0).
#include <cmath>
#include <mutex>
#include <string>

#include "mlmc_common.hpp"

using namespace aicdf;

// Device memory of the no-allocation entry point (mlmc_level_gbm_noalloc):
// the per-work-group partials of one level call, at most kMaxLevelBlocks
// work-groups of kSums doubles (192 KiB).  Each GPU the library runs on holds
// its own copy until the process ends.  Host code never passes `scratch`
// itself to a kernel or a copy (in host code the name is a stand-in, not a
// device address): the device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
static constexpr size_t kScratchDoubles = size_t(kMaxLevelBlocks) * kSums;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

struct GbmArgs {
  float S0, r_dt, r_2dt, sigma, sqrt_dt, dt, half_sig2, K, disc;
  double sqrt_dt_d;
  uint32_t level, nsteps;
  uint64_t n_paths, path_offset;
  uint32_t k0, k1, tag;
  const float* table;  // dyadic: 64 rows x 4 floats; geometric: the same, then
                       // 64 thresholds and 64 scales; constant: rows floats
  uint32_t rows;
  float inv_log2r;     // geometric: 1 / log2(r)
  int table_in_lds;
  uint32_t sparse;     // 1: one path per group of `group` lanes
  uint32_t group;      // lanes per path when sparse: min(64, 2^l / 2)
};

// A level of 2^l >= 4 steps runs one path per group of G = min(64, 2^l / 2)
// lanes (two or more steps per lane, so coarse steps stay within a lane) when
// its paths times G fit the lanes the GPU keeps resident (256 CUs x 2048):
// its time is then the serial time of 2^l / G steps instead of 2^l.  This
// includes one path per wavefront for up to 8192 paths at 2^l >= 128.
constexpr uint64_t kGbmGroupLanes = uint64_t(1) << 19;

// [[a, 0], [c, b]]: X' = a X, e' = c X + b e.
struct Lt2 {
  float a, c, b;
};

// y after x
__device__ __forceinline__ Lt2 lt2_mul(const Lt2& y, const Lt2& x) {
  return Lt2{y.a * x.a, fmaf(y.c, x.a, y.b * x.c), y.b * x.b};
}

// Ordered product over a group of G lanes (G a power of two, groups aligned
// within the wave), M_(G-1) ... M_0, delivered to the group's lane g = 0; a
// lane reads only lanes of its own group.
__device__ __forceinline__ Lt2 lt2_group_product(Lt2 m, int g, int G) {
  for (int d = 1; d < G; d <<= 1) {
    const Lt2 o{__shfl_down(m.a, d), __shfl_down(m.c, d), __shfl_down(m.b, d)};
    if ((g & (2 * d - 1)) == 0) m = lt2_mul(o, m);
  }
  return m;
}

// Approximate normal from the staged table (Algorithm 1 / Code 1).  Dyadic
// rows are zero-padded to four coefficients, so one cubic Horner pass gives
// the exact result of every degree.
template <int TAB>
__device__ __forceinline__ float approx_normal(float u, const float* tab, uint32_t rows, float inv_log2r) {
  if constexpr (TAB == 2) {
    // geometric rows (Theorem 2.5): ceil(log2(2t) / log2(r) - 1/64) is the
    // row or the one before it, one comparison with the FP32 threshold B_e
    // decides, then s = t / B_e; the same arithmetic as the streaming
    // transform
    const bool p = u < 0.5f;
    const float t = p ? u : 1.0f - u;
    const float t2 = 2.0f * t;
    const float x = __log2f(t2 < 0x1p-126f ? 0x1p-126f : t2) * inv_log2r;
    int e = int(fminf(fmaxf(ceilf(x - 0x1p-6f), 1.0f), float(rows - 1)));
    if (e < int(rows) - 1 && t < tab[256 + e]) ++e;
    if (t >= 0.5f) e = 0;
    const float s = t * tab[320 + e];
    const f32x4 c = reinterpret_cast<const f32x4*>(tab)[e];
    float z = fmaf(fmaf(fmaf(c[3], s, c[2]), s, c[1]), s, c[0]);
    return p ? z : -z;
  } else if constexpr (TAB == 0) {
    const bool p = u < 0.5f;
    const float ur = p ? u : 1.0f - u;
    const uint32_t e = min(126u - (__float_as_uint(ur) >> 23), rows - 1u);
    const float s = ur * __uint_as_float((128u + e) << 23);
    const f32x4 c = reinterpret_cast<const f32x4*>(tab)[e];
    float z = fmaf(fmaf(fmaf(c[3], s, c[2]), s, c[1]), s, c[0]);
    return p ? z : -z;
  } else {
    float x = fminf(fmaxf(u * float(rows), 0.0f), float(rows - 1));
    return tab[uint32_t(x)];
  }
}

// One scheme step X <- X (1 + inc) over h (= dt or 2 dt, r_h = r h):
// inc = r h + sigma dW, plus sigma^2 (dW^2 - h) / 2 for Milstein.
template <int SCHEME>
__device__ __forceinline__ float increment(const GbmArgs& a, float dW, float h, float r_h) {
  float inc = fmaf(a.sigma, dW, r_h);
  if (SCHEME == 1) inc = fmaf(a.half_sig2, fmaf(dW, dW, -h), inc);
  return inc;
}

template <int PAYOFF>
__device__ __forceinline__ float payoff(const GbmArgs& a, float X) {
  return PAYOFF == 0 ? X : a.disc * fmaxf(X - a.K, 0.0f);
}

// P(X~ + e) - P(X~) without cancellation.
template <int PAYOFF>
__device__ __forceinline__ float payoff_diff(const GbmArgs& a, float Xt, float e) {
  if (PAYOFF == 0) return e;
  const float m = Xt - a.K;
  if (m >= 0.0f && m + e >= 0.0f) return a.disc * e;
  if (m < 0.0f && m + e < 0.0f) return 0.0f;
  return a.disc * (fmaxf(m + e, 0.0f) - fmaxf(m, 0.0f));
}

// The step maps of steps [n0, n1) of one path (n0, n1 even), as products:
// fine f and coarse c.  The draws are those of the one-path-per-thread loop.
template <int KIND, int SCHEME, int TAB>
__device__ __forceinline__ void gbm_chunk(const GbmArgs& a, const float* tab, uint32_t plo, uint32_t phi, uint32_t n0,
                                          uint32_t n1, Lt2& f, Lt2& c) {
  f = Lt2{1.0f, 0.0f, 1.0f};
  c = Lt2{1.0f, 0.0f, 1.0f};
  if constexpr (KIND == AICDF_KIND_APPROX) {
    u32x4 w{};
    float dWprev = 0.0f;
    for (uint32_t n = n0; n < n1; ++n) {
      if ((n & 3u) == 0 || n == n0) w = philox4x32_10(n >> 2, plo, phi, a.tag, a.k0, a.k1);
      const float dW = a.sqrt_dt * approx_normal<TAB>(u24_from_word(w[n & 3u]), tab, a.rows, a.inv_log2r);
      f.a = fmaf(f.a, increment<SCHEME>(a, dW, a.dt, a.r_dt), f.a);
      if (n & 1u)
        c.a = fmaf(c.a, increment<SCHEME>(a, dWprev + dW, 2.0f * a.dt, a.r_2dt), c.a);
      else
        dWprev = dW;
    }
  } else if constexpr (KIND == AICDF_KIND_EXACT) {
    for (uint32_t n = n0; n < n1; n += 2) {
      const u32x4 w = philox4x32_10(n >> 1, plo, phi, a.tag, a.k0, a.k1);
      const float dW0 = float(exact_phi_inv(u53_from_words(w[0], w[1])) * a.sqrt_dt_d);
      const float dW1 = float(exact_phi_inv(u53_from_words(w[2], w[3])) * a.sqrt_dt_d);
      f.a = fmaf(f.a, increment<SCHEME>(a, dW0, a.dt, a.r_dt), f.a);
      f.a = fmaf(f.a, increment<SCHEME>(a, dW1, a.dt, a.r_dt), f.a);
      c.a = fmaf(c.a, increment<SCHEME>(a, dW0 + dW1, 2.0f * a.dt, a.r_2dt), c.a);
    }
  } else {
    for (uint32_t n = n0; n < n1; n += 2) {
      const u32x4 w = philox4x32_10(n >> 1, plo, phi, a.tag, a.k0, a.k1);
      float sh = 0.0f, st = 0.0f, sd = 0.0f;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double Z = exact_phi_inv(u53_from_words(w[2 * h], w[2 * h + 1]));
        const float Zt = approx_normal<TAB>(u24_from_word(w[2 * h]), tab, a.rows, a.inv_log2r);
        const float dWh = float(Z * a.sqrt_dt_d);
        const float dWt = a.sqrt_dt * Zt;
        const float d = float((Z - double(Zt)) * a.sqrt_dt_d);
        const float gh = increment<SCHEME>(a, dWh, a.dt, a.r_dt);
        float dg = a.sigma * d;
        if (SCHEME == 1) dg = fmaf(a.half_sig2 * d, dWh + dWt, dg);
        f.c = fmaf(dg, f.a, fmaf(f.c, gh, f.c));
        f.b = fmaf(f.b, gh, f.b);
        f.a = fmaf(f.a, increment<SCHEME>(a, dWt, a.dt, a.r_dt), f.a);
        sh += dWh;
        st += dWt;
        sd += d;
      }
      const float h2 = 2.0f * a.dt;
      const float gh = increment<SCHEME>(a, sh, h2, a.r_2dt);
      float dg = a.sigma * sd;
      if (SCHEME == 1) dg = fmaf(a.half_sig2 * sd, sh + st, dg);
      c.c = fmaf(dg, c.a, fmaf(c.c, gh, c.c));
      c.b = fmaf(c.b, gh, c.b);
      c.a = fmaf(c.a, increment<SCHEME>(a, st, h2, a.r_2dt), c.a);
    }
  }
}

// The approximation's table staged in LDS (when it fits), else read from
// global memory.
template <int TAB>
__device__ __forceinline__ const float* stage_table(const GbmArgs& a) {
  extern __shared__ f32x4 lds4[];
  if (!a.table_in_lds) return a.table;
  float* l = reinterpret_cast<float*>(lds4);
  const uint32_t nf = TAB == 0 ? 64u * 4u : TAB == 2 ? 64u * 6u : a.rows;
  for (uint32_t i = threadIdx.x; i < nf; i += kLevelBlock) l[i] = a.table[i];
  __syncthreads();
  return l;
}

// Work-group `bid` of the `nblk` work-groups of one level: its paths (a
// grid-stride loop over nblk work-groups), their sums into partials[bid].
template <int KIND, int SCHEME, int PAYOFF, int TAB, bool SPARSE>
__device__ __forceinline__ void gbm_level_block(const GbmArgs& a, const float* tab, double* __restrict__ partials,
                                                double* __restrict__ path_out, uint32_t bid, uint32_t nblk) {
  LevelAcc acc;
  const uint32_t nf = a.nsteps;
  if constexpr (SPARSE) {
    // one path per group of G lanes; lane g of a group takes steps
    // [g m, g m + m), m = 2^l / G (even)
    const int G = int(a.group);
    const int g = int(threadIdx.x) & (G - 1);
    const uint32_t m = nf / uint32_t(G);
    const uint64_t per_block = kLevelBlock / G;
    for (uint64_t base = uint64_t(bid) * per_block; base < a.n_paths; base += uint64_t(nblk) * per_block) {
      const uint64_t i = base + threadIdx.x / G;
      if (i >= a.n_paths) continue;  // uniform over each group
      const uint64_t P = a.path_offset + i;
      Lt2 f, c;
      gbm_chunk<KIND, SCHEME, TAB>(a, tab, uint32_t(P), uint32_t(P >> 32), g * m, g * m + m, f, c);
      f = lt2_group_product(f, g, G);
      c = lt2_group_product(c, g, G);
      if (g == 0) {
        float Y, Pf, Pc;
        const float Xf = a.S0 * f.a, Xc = a.S0 * c.a;
        if constexpr (KIND == AICDF_KIND_CORRECTION) {
          const float ef = a.S0 * f.c, ec = a.S0 * c.c;
          const float df = payoff_diff<PAYOFF>(a, Xf, ef);
          const float dc = payoff_diff<PAYOFF>(a, Xc, ec);
          Y = df - dc;
          Pf = payoff<PAYOFF>(a, Xf + ef);
          Pc = payoff<PAYOFF>(a, Xc + ec);
        } else {
          Pf = payoff<PAYOFF>(a, Xf);
          Pc = payoff<PAYOFF>(a, Xc);
          Y = Pf - Pc;
        }
        acc.add(double(Y), double(Pf), double(Pc));
        if (path_out) {
          path_out[3 * i] = double(Y);
          path_out[3 * i + 1] = double(Pf);
          path_out[3 * i + 2] = double(Pc);
        }
      }
    }
    block_reduce_store(acc, partials, bid);
    return;
  }
  const uint64_t stride = uint64_t(nblk) * kLevelBlock;
  for (uint64_t i = uint64_t(bid) * kLevelBlock + threadIdx.x; i < a.n_paths; i += stride) {
    const uint64_t P = a.path_offset + i;
    const uint32_t plo = uint32_t(P), phi = uint32_t(P >> 32);
    float Y, Pf, Pc;
    if constexpr (KIND == AICDF_KIND_APPROX) {
      float Xf = a.S0, Xc = a.S0, dWprev = 0.0f;
      for (uint32_t b = 0; b * 4 < nf; ++b) {
        const u32x4 w = philox4x32_10(b, plo, phi, a.tag, a.k0, a.k1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (b * 4 + q < nf) {
            const float dW = a.sqrt_dt * approx_normal<TAB>(u24_from_word(w[q]), tab, a.rows, a.inv_log2r);
            Xf = fmaf(Xf, increment<SCHEME>(a, dW, a.dt, a.r_dt), Xf);
            if (q & 1) {
              Xc = fmaf(Xc, increment<SCHEME>(a, dWprev + dW, 2.0f * a.dt, a.r_2dt), Xc);
            } else {
              dWprev = dW;
            }
          }
        }
      }
      Pf = payoff<PAYOFF>(a, Xf);
      Pc = a.level ? payoff<PAYOFF>(a, Xc) : 0.0f;
      Y = Pf - Pc;
    } else if constexpr (KIND == AICDF_KIND_EXACT) {
      float Xf = a.S0, Xc = a.S0;
      for (uint32_t b = 0; b * 2 < nf; ++b) {
        const u32x4 w = philox4x32_10(b, plo, phi, a.tag, a.k0, a.k1);
        const float dW0 = float(exact_phi_inv(u53_from_words(w[0], w[1])) * a.sqrt_dt_d);
        Xf = fmaf(Xf, increment<SCHEME>(a, dW0, a.dt, a.r_dt), Xf);
        if (nf > 1) {
          const float dW1 = float(exact_phi_inv(u53_from_words(w[2], w[3])) * a.sqrt_dt_d);
          Xf = fmaf(Xf, increment<SCHEME>(a, dW1, a.dt, a.r_dt), Xf);
          Xc = fmaf(Xc, increment<SCHEME>(a, dW0 + dW1, 2.0f * a.dt, a.r_2dt), Xc);
        }
      }
      Pf = payoff<PAYOFF>(a, Xf);
      Pc = a.level ? payoff<PAYOFF>(a, Xc) : 0.0f;
      Y = Pf - Pc;
    } else {
      // correction: approximate path + difference state, fine and coarse
      float Xf = a.S0, ef = 0.0f, Xc = a.S0, ec = 0.0f;
      for (uint32_t b = 0; b * 2 < nf; ++b) {
        const u32x4 w = philox4x32_10(b, plo, phi, a.tag, a.k0, a.k1);
        float sh = 0.0f, st = 0.0f, sd = 0.0f;  // coarse sums of dW^, dW~, d
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (b * 2 + h < nf) {
            const double Z = exact_phi_inv(u53_from_words(w[2 * h], w[2 * h + 1]));
            const float Zt = approx_normal<TAB>(u24_from_word(w[2 * h]), tab, a.rows, a.inv_log2r);
            const float dWh = float(Z * a.sqrt_dt_d);
            const float dWt = a.sqrt_dt * Zt;
            const float d = float((Z - double(Zt)) * a.sqrt_dt_d);
            const float gh = increment<SCHEME>(a, dWh, a.dt, a.r_dt);
            float dg = a.sigma * d;
            if (SCHEME == 1) dg = fmaf(a.half_sig2 * d, dWh + dWt, dg);
            ef = fmaf(Xf, dg, fmaf(ef, gh, ef));
            Xf = fmaf(Xf, increment<SCHEME>(a, dWt, a.dt, a.r_dt), Xf);
            sh += dWh;
            st += dWt;
            sd += d;
          }
        }
        if (nf > 1) {
          const float h2 = 2.0f * a.dt;
          const float gh = increment<SCHEME>(a, sh, h2, a.r_2dt);
          float dg = a.sigma * sd;
          if (SCHEME == 1) dg = fmaf(a.half_sig2 * sd, sh + st, dg);
          ec = fmaf(Xc, dg, fmaf(ec, gh, ec));
          Xc = fmaf(Xc, increment<SCHEME>(a, st, h2, a.r_2dt), Xc);
        }
      }
      const float df = payoff_diff<PAYOFF>(a, Xf, ef);
      const float dc = a.level ? payoff_diff<PAYOFF>(a, Xc, ec) : 0.0f;
      Y = df - dc;
      Pf = payoff<PAYOFF>(a, Xf + ef);
      Pc = a.level ? payoff<PAYOFF>(a, Xc + ec) : 0.0f;
    }
    acc.add(double(Y), double(Pf), double(Pc));
    if (path_out) {
      path_out[3 * i] = double(Y);
      path_out[3 * i + 1] = double(Pf);
      path_out[3 * i + 2] = double(Pc);
    }
  }
  block_reduce_store(acc, partials, bid);
}

template <int KIND, int SCHEME, int PAYOFF, int TAB, bool SPARSE>
__global__ __launch_bounds__(kLevelBlock) void gbm_level_kernel(GbmArgs a, double* __restrict__ partials,
                                                               double* __restrict__ path_out) {
  const float* tab = KIND != AICDF_KIND_EXACT ? stage_table<TAB>(a) : a.table;
  gbm_level_block<KIND, SCHEME, PAYOFF, TAB, SPARSE>(a, tab, partials, path_out, blockIdx.x, gridDim.x);
}

// The level jobs of one batched call: the arguments of each job's level call
// and the work-group spans (job j owns [start[j], start[j+1])).
struct GbmBatch {
  GbmArgs job[kMaxJobs];
  uint32_t start[kMaxJobs + 1];
  uint32_t n_jobs;
};
// kernel arguments are limited to 4 KiB (with the pointer that follows)
static_assert(sizeof(GbmBatch) + 64 <= 4096, "batched GBM arguments exceed the kernel argument limit");

// KSET 0: EXACT jobs only; 1: APPROX jobs only; 2: any kinds.  Each
// work-group finds its job (a wave-uniform scan of at most kMaxJobs spans)
// and runs that job's level code on its share of the job's paths.
template <int KSET, int SCHEME, int PAYOFF, int TAB>
__global__ __launch_bounds__(kLevelBlock) void gbm_levels_kernel(GbmBatch b, double* __restrict__ partials) {
  uint32_t j = 0;
  while (j + 1 < b.n_jobs && blockIdx.x >= b.start[j + 1]) ++j;
  const GbmArgs a = b.job[j];
  const uint32_t bid = blockIdx.x - b.start[j], nblk = b.start[j + 1] - b.start[j];
  double* part = partials + size_t(b.start[j]) * kSums;
  const int kind = int(a.tag >> 8);
  if constexpr (KSET == 0) {
    if (a.sparse)
      gbm_level_block<AICDF_KIND_EXACT, SCHEME, PAYOFF, TAB, true>(a, a.table, part, nullptr, bid, nblk);
    else
      gbm_level_block<AICDF_KIND_EXACT, SCHEME, PAYOFF, TAB, false>(a, a.table, part, nullptr, bid, nblk);
  } else {
    const float* tab = kind != AICDF_KIND_EXACT ? stage_table<TAB>(a) : a.table;
    if (KSET == 1 || kind == AICDF_KIND_APPROX) {
      if (a.sparse)
        gbm_level_block<AICDF_KIND_APPROX, SCHEME, PAYOFF, TAB, true>(a, tab, part, nullptr, bid, nblk);
      else
        gbm_level_block<AICDF_KIND_APPROX, SCHEME, PAYOFF, TAB, false>(a, tab, part, nullptr, bid, nblk);
    } else if constexpr (KSET == 2) {
      if (kind == AICDF_KIND_CORRECTION) {
        if (a.sparse)
          gbm_level_block<AICDF_KIND_CORRECTION, SCHEME, PAYOFF, TAB, true>(a, tab, part, nullptr, bid, nblk);
        else
          gbm_level_block<AICDF_KIND_CORRECTION, SCHEME, PAYOFF, TAB, false>(a, tab, part, nullptr, bid, nblk);
      } else {
        if (a.sparse)
          gbm_level_block<AICDF_KIND_EXACT, SCHEME, PAYOFF, TAB, true>(a, tab, part, nullptr, bid, nblk);
        else
          gbm_level_block<AICDF_KIND_EXACT, SCHEME, PAYOFF, TAB, false>(a, tab, part, nullptr, bid, nblk);
      }
    }
  }
}

template <int KSET, int SCHEME, int PAYOFF>
void launch_batch_tab(int tab, const GbmBatch& b, unsigned grid, size_t lds, hipStream_t s, double* p) {
  if (tab == 0 || KSET == 0)
    hipLaunchKernelGGL((gbm_levels_kernel<KSET, SCHEME, PAYOFF, 0>), dim3(grid), dim3(kLevelBlock), lds, s, b, p);
  else if (tab == 2)
    hipLaunchKernelGGL((gbm_levels_kernel<KSET, SCHEME, PAYOFF, 2>), dim3(grid), dim3(kLevelBlock), lds, s, b, p);
  else
    hipLaunchKernelGGL((gbm_levels_kernel<KSET, SCHEME, PAYOFF, 1>), dim3(grid), dim3(kLevelBlock), lds, s, b, p);
}

template <int KSET>
void launch_batch(int scheme, int payoff, int tab, const GbmBatch& b, unsigned grid, size_t lds, hipStream_t s,
                  double* p) {
  if (scheme == 0 && payoff == 0) launch_batch_tab<KSET, 0, 0>(tab, b, grid, lds, s, p);
  if (scheme == 0 && payoff == 1) launch_batch_tab<KSET, 0, 1>(tab, b, grid, lds, s, p);
  if (scheme == 1 && payoff == 0) launch_batch_tab<KSET, 1, 0>(tab, b, grid, lds, s, p);
  if (scheme == 1 && payoff == 1) launch_batch_tab<KSET, 1, 1>(tab, b, grid, lds, s, p);
}

template <int KIND, int SCHEME, int PAYOFF, int TAB>
void launch(const GbmArgs& a, unsigned grid, size_t lds, hipStream_t s, double* partials, double* path_out) {
  if (a.sparse)
    hipLaunchKernelGGL((gbm_level_kernel<KIND, SCHEME, PAYOFF, TAB, true>), dim3(grid), dim3(kLevelBlock), lds, s,
                       a, partials, path_out);
  else
    hipLaunchKernelGGL((gbm_level_kernel<KIND, SCHEME, PAYOFF, TAB, false>), dim3(grid), dim3(kLevelBlock), lds, s,
                       a, partials, path_out);
}

template <int KIND, int SCHEME, int PAYOFF>
void launch_tab(int tab, const GbmArgs& a, unsigned grid, size_t lds, hipStream_t s, double* p, double* po) {
  if (tab == 0)
    launch<KIND, SCHEME, PAYOFF, 0>(a, grid, lds, s, p, po);
  else if (tab == 2)
    launch<KIND, SCHEME, PAYOFF, 2>(a, grid, lds, s, p, po);
  else
    launch<KIND, SCHEME, PAYOFF, 1>(a, grid, lds, s, p, po);
}

template <int KIND>
void launch_kind(int scheme, int payoff, int tab, const GbmArgs& a, unsigned grid, size_t lds, hipStream_t s,
                 double* p, double* po) {
  if (scheme == 0 && payoff == 0) launch_tab<KIND, 0, 0>(tab, a, grid, lds, s, p, po);
  if (scheme == 0 && payoff == 1) launch_tab<KIND, 0, 1>(tab, a, grid, lds, s, p, po);
  if (scheme == 1 && payoff == 0) launch_tab<KIND, 1, 0>(tab, a, grid, lds, s, p, po);
  if (scheme == 1 && payoff == 1) launch_tab<KIND, 1, 1>(tab, a, grid, lds, s, p, po);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the device's first
// call, with that device current).
aicdf_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(AICDF_EINVAL, "device %d beyond the supported %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(AICDF_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return AICDF_OK;
}

// scratch_partials: when non-NULL the level's partials go there and the sums
// to out.dev with no workspace (nothing allocated, no lock); else the
// per-stream workspace is used.
// Checks one level's arguments and fills its kernel arguments, table kind,
// LDS bytes and work-group count (the launch shape of its level call).
aicdf_status setup_gbm(const aicdf_gbm_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                       const aicdf_table* approx, uint64_t seed, uint64_t path_offset, int dev, GbmArgs& a,
                       int& tab, size_t& lds, unsigned& grid) {
  if (level > 20) return fail(AICDF_ERANGE, "level %u > 20", level);
  if (kind < 0 || kind > 2) return fail(AICDF_EINVAL, "kind must be 0, 1 or 2");
  if (kind != AICDF_KIND_EXACT && !approx) return fail(AICDF_EINVAL, "the approximate kinds need a table");
  if (n_paths > (uint64_t(1) << 40)) return fail(AICDF_ERANGE, "n_paths > 2^40");
  if (path_offset + n_paths < path_offset) return fail(AICDF_ERANGE, "path_offset + n_paths overflows");
  if (approx && kind != AICDF_KIND_EXACT && approx->device != dev)
    return fail(AICDF_EINVAL, "table lives on device %d, current device is %d", approx->device, dev);

  const uint32_t nf = 1u << level;
  const double dt = prm->T / nf;
  a = GbmArgs{};
  a.S0 = float(prm->S0);
  a.r_dt = float(prm->r * dt);
  a.r_2dt = float(prm->r * 2.0 * dt);
  a.sigma = float(prm->sigma);
  a.sqrt_dt = float(std::sqrt(dt));
  a.dt = float(dt);
  a.half_sig2 = float(0.5 * prm->sigma * prm->sigma);
  a.K = float(prm->K);
  a.disc = float(std::exp(-prm->r * prm->T));
  a.sqrt_dt_d = std::sqrt(dt);
  a.level = level;
  a.nsteps = nf;
  a.n_paths = n_paths;
  a.path_offset = path_offset;
  a.k0 = uint32_t(seed);
  a.k1 = uint32_t(seed >> 32);
  a.tag = level | (uint32_t(kind) << 8);
  tab = 0;
  lds = 0;
  if (kind != AICDF_KIND_EXACT) {
    tab = approx->kind == 1 ? 0 : approx->kind == 2 ? 2 : 1;
    if (tab == 2) a.inv_log2r = float(1.0 / std::log2(approx->r));
    if (tab == 1 && approx->coef_t == AICDF_F64)
      return fail(AICDF_EDTYPE, "the fused levels use FP32 arithmetic: the constant table must not be F64");
    a.table = static_cast<const float*>(approx->dev);
    a.rows = approx->rows;
    const size_t bytes = tab == 0 ? 64 * 16 : tab == 2 ? 64 * 24 : size_t(approx->rows) * 4;
    a.table_in_lds = bytes <= 64 * 1024;
    lds = a.table_in_lds ? bytes : 0;
  }
  a.group = nf >= 4 ? (nf / 2 < 64 ? nf / 2 : 64) : 0u;
  a.sparse = (a.group && n_paths * a.group <= kGbmGroupLanes) ? 1u : 0u;
  const uint64_t per_block = a.sparse ? kLevelBlock / a.group : kLevelBlock;
  const uint64_t need = (n_paths + per_block - 1) / per_block;
  grid = unsigned(need < uint64_t(kMaxLevelBlocks) ? need : kMaxLevelBlocks);
  return AICDF_OK;
}

aicdf_status check_gbm_params(const aicdf_gbm_params* prm) {
  if (!prm) return fail(AICDF_EINVAL, "params must be non-NULL");
  if (prm->scheme < 0 || prm->scheme > 1 || prm->payoff < 0 || prm->payoff > 1)
    return fail(AICDF_EINVAL, "scheme and payoff must be 0 or 1");
  if (!(prm->T > 0.0) || !(prm->sigma >= 0.0) || !std::isfinite(prm->S0) || !std::isfinite(prm->r))
    return fail(AICDF_EINVAL, "need T > 0, sigma >= 0, finite S0 and r");
  return AICDF_OK;
}

aicdf_status gbm_level(const aicdf_gbm_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                       const aicdf_table* approx, uint64_t seed, uint64_t path_offset, const LevelOut& out,
                       double* path_out, void* stream, bool no_alloc = false) {
  aicdf_status st = check_gbm_params(prm);
  if (st != AICDF_OK) return st;
  st = check_level_out(out);
  if (st != AICDF_OK) return st;
  if (level > 20) return fail(AICDF_ERANGE, "level %u > 20", level);
  if (kind < 0 || kind > 2) return fail(AICDF_EINVAL, "kind must be 0, 1 or 2");
  if (kind != AICDF_KIND_EXACT && !approx) return fail(AICDF_EINVAL, "the approximate kinds need a table");
  if (n_paths == 0) return no_alloc ? reduce_partials_to(nullptr, 0, 0.0, out.dev, static_cast<hipStream_t>(stream))
                                    : empty_level(static_cast<hipStream_t>(stream), out);
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  GbmArgs a;
  int tab = 0;
  size_t lds = 0;
  unsigned grid = 0;
  st = setup_gbm(prm, level, n_paths, kind, approx, seed, path_offset, dev, a, tab, lds, grid);
  if (st != AICDF_OK) return st;

  auto s = static_cast<hipStream_t>(stream);
  if (no_alloc) {
    double* partials = nullptr;
    st = scratch_address(dev, &partials);
    if (st != AICDF_OK) return st;
    if (size_t(grid) * kSums > kScratchDoubles)
      return fail(AICDF_ERANGE, "%u work-groups need %zu doubles of scratch, the maximum is %zu", grid,
                  size_t(grid) * kSums, kScratchDoubles);
    if (kind == AICDF_KIND_EXACT)
      launch_kind<AICDF_KIND_EXACT>(prm->scheme, prm->payoff, 0, a, grid, 0, s, partials, path_out);
    else if (kind == AICDF_KIND_APPROX)
      launch_kind<AICDF_KIND_APPROX>(prm->scheme, prm->payoff, tab, a, grid, lds, s, partials, path_out);
    else
      launch_kind<AICDF_KIND_CORRECTION>(prm->scheme, prm->payoff, tab, a, grid, lds, s, partials, path_out);
    AICDF_HIP(hipGetLastError());
    return reduce_partials_to(partials, grid, double(n_paths), out.dev, s);
  }
  Workspace* ws = nullptr;
  st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  st = begin_level(ws, s, out);
  if (st != AICDF_OK) return st;
  if (kind == AICDF_KIND_EXACT)
    launch_kind<AICDF_KIND_EXACT>(prm->scheme, prm->payoff, 0, a, grid, 0, s, ws->partials, path_out);
  else if (kind == AICDF_KIND_APPROX)
    launch_kind<AICDF_KIND_APPROX>(prm->scheme, prm->payoff, tab, a, grid, lds, s, ws->partials, path_out);
  else
    launch_kind<AICDF_KIND_CORRECTION>(prm->scheme, prm->payoff, tab, a, grid, lds, s, ws->partials, path_out);
  AICDF_HIP(hipGetLastError());
  return finish_level(ws, grid, s, double(n_paths), out);
}

}  // namespace

extern "C" aicdf_status mlmc_level_gbm(const aicdf_gbm_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                                       const aicdf_table* approx, uint64_t seed, uint64_t path_offset,
                                       aicdf_level_sums* out, double* path_out, void* stream) {
  if (!out) return fail(AICDF_EINVAL, "out must be non-NULL");
  return gbm_level(prm, level, n_paths, kind, approx, seed, path_offset, LevelOut{out, nullptr}, path_out, stream);
}

extern "C" aicdf_status mlmc_level_gbm_async(const aicdf_gbm_params* prm, uint32_t level, uint64_t n_paths,
                                             int32_t kind, const aicdf_table* approx, uint64_t seed,
                                             uint64_t path_offset, double* sums_dev, double* path_out, void* stream) {
  if (!sums_dev) return fail(AICDF_EINVAL, "sums_dev must be non-NULL");
  return gbm_level(prm, level, n_paths, kind, approx, seed, path_offset, LevelOut{nullptr, sums_dev}, path_out,
                   stream);
}

extern "C" aicdf_status mlmc_level_gbm_noalloc(const aicdf_gbm_params* prm, uint32_t level, uint64_t n_paths,
                                               int32_t kind, const aicdf_table* approx, uint64_t seed,
                                               uint64_t path_offset, double* sums_dev, double* path_out,
                                               void* stream) {
  if (!sums_dev) return fail(AICDF_EINVAL, "sums_dev must be non-NULL");
  return gbm_level(prm, level, n_paths, kind, approx, seed, path_offset, LevelOut{nullptr, sums_dev}, path_out,
                   stream, true);
}

extern "C" aicdf_status mlmc_levels_gbm(const aicdf_gbm_params* prm, const aicdf_level_job* jobs, uint32_t n_jobs,
                                        const aicdf_table* approx, uint64_t seed, double* sums_dev, void* stream) {
  aicdf_status st = check_gbm_params(prm);
  if (st != AICDF_OK) return st;
  if (n_jobs == 0) return ok();
  if (!jobs || !sums_dev) return fail(AICDF_EINVAL, "jobs and sums_dev must be non-NULL");
  if (n_jobs > uint32_t(kMaxJobs)) return fail(AICDF_ERANGE, "%u jobs > %d", n_jobs, kMaxJobs);
  if (reinterpret_cast<uintptr_t>(sums_dev) & 7u) return fail(AICDF_EINVAL, "sums_dev must be 8-byte aligned");
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  GbmBatch b{};
  JobSpans sp{};
  b.n_jobs = sp.n_jobs = n_jobs;
  bool any_exact = false, any_approx = false, any_corr = false;
  int tab = -1;
  size_t lds = 0;
  uint32_t total = 0;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    const aicdf_level_job& jb = jobs[j];
    int t = 0;
    size_t l = 0;
    unsigned g = 0;
    st = setup_gbm(prm, jb.level, jb.n_paths, jb.kind, approx, seed, jb.path_offset, dev, b.job[j], t, l, g);
    if (st != AICDF_OK) {
      const std::string msg = aicdf_last_error();
      return fail(st, "job %u: %s", j, msg.c_str());
    }
    if (jb.n_paths == 0) g = 0;
    if (jb.kind != AICDF_KIND_EXACT) {
      tab = t;
      lds = l;
    }
    any_exact |= jb.kind == AICDF_KIND_EXACT;
    any_approx |= jb.kind == AICDF_KIND_APPROX;
    any_corr |= jb.kind == AICDF_KIND_CORRECTION;
    sp.start[j] = b.start[j] = total;
    sp.n_paths[j] = double(jb.n_paths);
    total += g;
  }
  sp.start[n_jobs] = b.start[n_jobs] = total;
  auto s = static_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  st = get_batch_buffers(ws);
  if (st != AICDF_OK) return st;
  if (total > 0) {
    if (!any_approx && !any_corr)
      launch_batch<0>(prm->scheme, prm->payoff, 0, b, total, 0, s, ws->batch_partials);
    else if (!any_exact && !any_corr)
      launch_batch<1>(prm->scheme, prm->payoff, tab, b, total, lds, s, ws->batch_partials);
    else
      launch_batch<2>(prm->scheme, prm->payoff, tab, b, total, lds, s, ws->batch_partials);
    AICDF_HIP(hipGetLastError());
  }
  return reduce_batch(ws->batch_partials, sp, nullptr, sums_dev, s);
}
