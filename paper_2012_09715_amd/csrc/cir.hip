// Fused MLMC level of the CIR process with exact-in-law non-central
// chi-squared transitions (Section 5.2).  One path per thread; per step n:
//   lambda_n = v_n e^(-kappa delta) / c,  v_(n+1) = c C_nu^-1(U_n; lambda_n),
// with C_nu^-1 the exact FP64 inverse (EXACT), an FP32 approximation
// (APPROX), or both on one draw (CORRECTION).  Two approximations:
//   APX_SURROGATE  P~ = MLP(D(U), g(log lambda)), x = lambda + nu +
//                  2 sqrt(lambda+nu) P~, clamped at 0.  The network call is a
//                  wave-wide matrix-core routine, so all 64 lanes step
//                  together.  Outside the trained log-lambda range the
//                  network is evaluated at the range's nearer end (counted
//                  as fallbacks): below it (lambda = 0 included, after a step
//                  clamped at 0) P depends on lambda only through O(lambda)
//                  terms, above it (e^10 = 22026 for the benchmark's
//                  network) P is within O(lambda^-1/2) of its Gaussian
//                  limit; the correction level removes the bias either way.
//                  No exact inverse in the approximate kind: its registers
//                  would halve the waves the level keeps per SIMD.
//   APX_POLY1/3    Section 5.1's piecewise-polynomial approximation (two
//                  dyadic half tables per knot, linear interpolation in
//                  sqrt(y)), clamped at 0; the table is staged in LDS.
//   APX_SANKARAN   Section 5.1's comparator (sankaran_x), clamped at 0.
//   APX_EM         the truncated Euler-Maruyama step of Section 5.2 (the
//                  Gaussian scheme the approximations are compared with):
//                  v' = v + kappa (theta - v) delta + xi sqrt(|v| delta) Z,
//                  Z = Phi^-1(u24) in FP64, the state in FP32 (may go
//                  negative; |v| under the root).
// A fourth kind, TWOWAY, runs the exact and the approximate fine paths on the
// same draws (as CORRECTION) and returns Y = P^_f - P~_f, P_f = P^_f,
// P_c = P~_f: the two-way difference at one time step (Figure 4b).
// Launch shape.  Calls with exact inversions and few paths (the high levels
// of an MLMC allocation, where a level's time is the serial time of one
// path) run one path per wavefront: all 64 lanes follow the same path and
// evaluate each exact inverse together (ncx2_wave.hpp), and lane 0 keeps the
// sums; no path waits for the root iterations of 63 others.  Every other
// call runs one path per thread; the crossover is a cost model (below).
// The coarse path of level l is the fine path
// observed at even steps (exact in law), so only the functional differs:
//   FUNC 0  P = v_T
//   FUNC 1  P = trapezoidal time average on the level's grid.
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "chi2_device.hpp"
#include "mlmc_common.hpp"
#include "mlp_device.hpp"
#include "ncx2_device.hpp"
#include "ncx2_wave.hpp"

using namespace aicdf;

namespace {

constexpr int APX_SURROGATE = 0, APX_POLY1 = 1, APX_POLY3 = 3, APX_EM = 4, APX_SANKARAN = 5;
constexpr int KIND_TWOWAY = 3;
constexpr uint32_t kMaxLdsRows = 2048;  // 32 KiB of chi-squared table rows

struct CirArgs {
  double nu, c, decay, v0;
  float nuf, cf, decayf, v0f;
  float lamf;      // decay / c: lambda of the next step is lamf times the variance
  float g_a, g_b;  // surrogate feature before clamping: g = g_a log2(lambda) + g_b
  uint32_t level, nsteps;
  uint64_t n_paths, path_offset;
  uint32_t k0, k1, tag;
  float kdt, theta, xi_sqdt;  // APX_EM: kappa delta, theta, xi sqrt(delta)
  Chi2Geom geo;         // APX_POLY*: table geometry
  uint32_t table_rows;  // APX_POLY*: rows staged in LDS
  uint32_t sparse;      // 1: one path per wavefront
};

// Launch shape of the exact, correction and two-way kinds.  One path per
// thread gives a call of n paths n/64 waves, each as slow per step as its
// slowest lane's root iteration; one path per wavefront gives n waves, each
// evaluating one inverse with all its lanes, and costs about n/W times one
// wave's serial time once the n waves exceed the W the GPU keeps resident.
// The ratio r of the two per-step times grows with lambda (a thread's sweep
// has ~18 sqrt(mu) terms and lanes diverge; the wave splits the sweep 64
// ways), so a call runs one path per wavefront below n* = W r(lambda), with
// lambda at the process level max(v0, theta) and r measured on MI355X for the
// exact kind (nu = 0.89, levels 0..10; the last two points extrapolated):
constexpr float kShapeRatio[12] = {4.0f, 4.8f, 6.0f, 7.6f, 9.1f, 10.5f, 11.7f, 14.1f, 21.8f, 33.3f, 45.0f, 57.0f};
constexpr int kShapeLog2Lo = 2;  // kShapeRatio[k] at log2 lambda = k + 2
// n* is kept within [2049, 2^17]: calls of at most 2048 paths always run one
// path per wavefront and calls of 2^17 or more one path per thread.
constexpr uint64_t kSparseAlways = 2048, kDenseAlways = uint64_t(1) << 17;

float shape_ratio(double lam) {
  const double x = std::log2(std::fmax(lam, 1e-300)) - kShapeLog2Lo;
  if (!(x > 0.0)) return kShapeRatio[0];
  if (x >= 11.0) return kShapeRatio[11];
  const int k = int(x);
  const float f = float(x - k);
  return kShapeRatio[k] + f * (kShapeRatio[k + 1] - kShapeRatio[k]);
}

// Waves of `kernel` the current device keeps resident (blocks per CU from the
// occupancy calculator x CUs x 4), cached per (device, kernel, LDS bytes).
aicdf_status resident_waves(const void* kernel, size_t lds, uint64_t* waves) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, uint64_t> cache;
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, kernel, lds);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *waves = it->second;
    return AICDF_OK;
  }
  int blocks = 0, cus = 0;
  AICDF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, kLevelBlock, lds));
  AICDF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  *waves = uint64_t(blocks > 0 ? blocks : 1) * uint64_t(cus > 0 ? cus : 1) * (kLevelBlock / 64);
  cache[key] = *waves;
  return AICDF_OK;
}

__device__ __forceinline__ float dyadic_w16(float u, const f32x4* __restrict__ tab) {
  const bool p = u < 0.5f;
  const float ur = p ? u : 1.0f - u;
  const uint32_t e = min(126u - (__float_as_uint(ur) >> 23), 15u);
  const float s = ur * __uint_as_float((128u + e) << 23);
  const f32x4 c = tab[e];
  const float z = fmaf(fmaf(fmaf(c[3], s, c[2]), s, c[1]), s, c[0]);
  return p ? z : -z;
}

// Trapezoidal sums of one path: fine over every node, coarse over even nodes.
struct FuncAcc {
  double fine = 0.0, coarse = 0.0;
  __device__ __forceinline__ void node(uint32_t k, uint32_t N, double v) {
    const double wt = (k == 0 || k == N) ? 0.5 : 1.0;
    fine += wt * v;
    if ((k & 1u) == 0) coarse += wt * v;
  }
  template <int FUNC>
  __device__ __forceinline__ void result(uint32_t level, uint32_t N, double vN, double& Pf, double& Pc) const {
    if (FUNC == 0) {
      Pf = vN;
      Pc = level ? vN : 0.0;
    } else {
      Pf = fine / N;
      Pc = level ? coarse / (N / 2) : 0.0;
    }
  }
};

// The exact inverse behind a function call, for the one-path-per-thread
// kernels that also run an approximation: inlined, its registers add to those
// the approximation keeps live (the network's weight fragments above all) and
// leave one wave per SIMD; behind a call the kernel needs the larger of the
// two.  (One path per wavefront the network reads its weights from LDS and
// the inverse stays inline: there a call's register saves cost more.)
// lga1 = log Gamma(nu/2 + 1), taken once per thread instead of once per
// inverse (the library log-gamma is a long serial chain).
__device__ __noinline__ double ncx2_icdf_call(double u, double nu, double lam, double x0, double lga1) {
  return ncx2_icdf(u, nu, lam, nullptr, x0, lga1);
}
__device__ __noinline__ double ncx2_icdf_wave_call(double u, double nu, double lam, double x0, double lga1) {
  return ncx2_icdf_wave(u, nu, lam, x0, lga1);
}

template <bool SPARSE, bool CALL>
__device__ __forceinline__ double exact_inverse(double u, double nu, double lam, double x0, double lga1) {
  if (CALL) return SPARSE ? ncx2_icdf_wave_call(u, nu, lam, x0, lga1) : ncx2_icdf_call(u, nu, lam, x0, lga1);
  return SPARSE ? ncx2_icdf_wave(u, nu, lam, x0, lga1) : ncx2_icdf(u, nu, lam, nullptr, x0, lga1);
}

// Regrouping of the paths between steps in the kinds with the exact inverse
// (one path per thread).  The exact inverse's cost per step grows with lambda
// (its sweeps visit about 18 sqrt(lambda/2) + 32 terms; small lambda needs a
// third evaluation), and a wave runs as long as its dearest lane.  Every
// kRegroupEvery steps the work-group ranks its 256 paths by the exact path's
// current v (lambda is v times a per-level constant) and moves them through
// LDS so that each wave holds 64 paths of neighbouring lambda.  Which wave
// takes which quarter of the order rotates with the regrouping and the
// work-group, so that no SIMD keeps the dearest quarter.  A path's arithmetic
// does not depend on the lane that runs it, and its results go back to its own
// lane before the sums: values and sums are those of the loop without
// regrouping, bit for bit.  kRegroupEvery is even: the Philox block of a pair
// of steps is drawn at the even step, after the move.
constexpr uint32_t kRegroupEvery = 4;
constexpr int kRegroupRows = 6;  // carried doubles: v, two trapezoid sums, per path (exact and approximate)
static_assert(kLevelBlock == 256 && kRegroupEvery % 2 == 0, "regrouping assumes four waves and step pairs");

struct RegroupLds {
  __align__(16) uint32_t key[kLevelBlock];
  uint32_t sid[kLevelBlock];
  double st[kRegroupRows][kLevelBlock];
};

// One LDS area per kernel that regroups (a function-scope static: kernels
// that never call this do not allocate it).
__device__ __forceinline__ RegroupLds& regroup_lds() {
  __shared__ RegroupLds R;
  return R;
}

// Moves this lane's path (block-local index sid and NST carried doubles, st[0]
// = v of the exact path) to lane dst of the order and takes the path that
// lands on this lane.  Keys are unique (the FP32 bits of v, order-preserving
// for v >= 0, with the low 8 bits replaced by the lane), so the ranks are a
// permutation whatever the values (NaN included).
template <int NST>
__device__ __forceinline__ void regroup(uint32_t rot, uint32_t& sid, double (&st)[NST]) {
  static_assert(NST <= kRegroupRows, "too many carried values");
  RegroupLds& R = regroup_lds();
  const uint32_t t = threadIdx.x;
  const uint32_t key = (__float_as_uint(float(st[0])) & ~0xFFu) | t;
  R.key[t] = key;
  __syncthreads();
  uint32_t r = 0;
  for (int j = 0; j < kLevelBlock; j += 4) {
    const u32x4 k = *reinterpret_cast<const u32x4*>(&R.key[j]);
    r += (k[0] < key ? 1u : 0u) + (k[1] < key ? 1u : 0u) + (k[2] < key ? 1u : 0u) + (k[3] < key ? 1u : 0u);
  }
  const uint32_t dst = ((((r >> 6) + rot) & 3u) << 6) | (r & 63u);
  R.sid[dst] = sid;
#pragma unroll
  for (int q = 0; q < NST; ++q) R.st[q][dst] = st[q];
  __syncthreads();
  sid = R.sid[t];
#pragma unroll
  for (int q = 0; q < NST; ++q) st[q] = R.st[q][t];
}

// Returns the three results of the path this lane ran to the lane of its
// block-local index sid (the first barrier ends the last regrouping's reads).
__device__ __forceinline__ void regroup_return(uint32_t sid, double& y, double& pf, double& pc) {
  RegroupLds& R = regroup_lds();
  __syncthreads();
  R.st[0][sid] = y;
  R.st[1][sid] = pf;
  R.st[2][sid] = pc;
  __syncthreads();
  y = R.st[0][threadIdx.x];
  pf = R.st[1][threadIdx.x];
  pc = R.st[2][threadIdx.x];
}

// Static LDS of a level work-group: the surrogate's staged parameters, the
// per-wave exchange of the one-sample network call, W2 (one path per
// wavefront only: W2 = true), the 16-row cubic table of the network's input
// feature, and the block's fallback counts.
template <bool W2>
struct CirLds {
  MlpLds L;
  MlpXchg xch[kLevelBlock / 64];
  __align__(16) uint16_t w2s[W2 ? kHidden * kW2Stride : 8];
  f32x4 tab[16];
  unsigned long long fbs[kLevelBlock];
};

// Work-group `bid` of the `nblk` work-groups of one level: its paths (a
// grid-stride loop over nblk work-groups), their sums into partials[bid],
// its fallbacks added to *fallbacks.  ctab: the dynamic LDS of the
// chi-squared table (APX_POLY*).
template <int KIND, int FUNC, int APX, bool SPARSE, bool W2>
__device__ __forceinline__ void cir_level_block(const CirArgs& a, const float* __restrict__ params,
                                                const uint16_t* __restrict__ w2b, const f32x4* __restrict__ wtab,
                                                double* __restrict__ partials, double* __restrict__ path_out,
                                                unsigned long long* __restrict__ fallbacks, uint32_t bid,
                                                uint32_t nblk, CirLds<W2>& S, f32x4* __restrict__ ctab) {
  constexpr bool kExact = KIND != AICDF_KIND_APPROX;
  constexpr bool kApx = KIND != AICDF_KIND_EXACT;
  constexpr bool kSurr = kApx && APX == APX_SURROGATE;
  constexpr bool kPoly = kApx && (APX == APX_POLY1 || APX == APX_POLY3);
  constexpr bool kEm = kApx && APX == APX_EM;
  constexpr bool kSank = kApx && APX == APX_SANKARAN;
  constexpr bool kCall = !SPARSE && (kSurr || kEm || kSank);
  static_assert(!(SPARSE && kSurr) || W2, "one path per wavefront with the surrogate needs W2 in LDS");
  MlpLds& L = S.L;
  MlpXchg* xch = S.xch;
  uint16_t* w2s = S.w2s;
  f32x4* tab = S.tab;
  bf16x8 A[2][4];
  if (kSurr) {
    mlp_stage_params(L, params, threadIdx.x, kLevelBlock);
    if (threadIdx.x < 16) tab[threadIdx.x] = wtab[threadIdx.x];
    if (SPARSE) mlp_stage_w2(w2s, w2b, threadIdx.x, kLevelBlock);
    __syncthreads();
    // one path per wavefront: the W2 fragments come from LDS at each call,
    // which leaves the wave-cooperative exact inverse its registers
    if (!SPARSE) mlp_load_w2(w2b, A);
  }
  if (kPoly) {
    for (uint32_t r = threadIdx.x; r < a.table_rows; r += kLevelBlock) ctab[r] = wtab[r];
    __syncthreads();
  }
  LevelAcc acc;
  unsigned long long fb = 0;
  const uint32_t N = a.nsteps;
  const double lga1 = kExact ? ncx2_lgamma(0.5 * a.nu + 1.0) : 0.0;
  const uint32_t per_block = SPARSE ? kLevelBlock / 64 : kLevelBlock;
  const uint32_t slot = SPARSE ? threadIdx.x / 64 : threadIdx.x;
  const bool lead = SPARSE ? (threadIdx.x % 64) == 0 : true;
  constexpr bool kRegroup = kExact && !SPARSE;
  for (uint64_t base = uint64_t(bid) * per_block; base < a.n_paths; base += uint64_t(nblk) * per_block) {
    const uint64_t i = base + slot;
    const bool act = lead && i < a.n_paths;   // lanes that keep the sums
    const bool work = SPARSE ? i < a.n_paths : true;  // wave-uniform when SPARSE
    uint32_t sid = slot;  // block-local index of the path this lane runs (moves when regrouped)
    bool cact = act;      // that path is one of the call's
    uint64_t P = a.path_offset + i;
    uint32_t plo = uint32_t(P), phi = uint32_t(P >> 32);
    double ve = a.v0;
    float vs = a.v0f;
    FuncAcc fe, fs;
    if (FUNC == 1) {
      fe.node(0, N, ve);
      fs.node(0, N, double(vs));
    }
    u32x4 w{};
    for (uint32_t n = 0; n < N; ++n) {
      if (kRegroup && n != 0 && n % kRegroupEvery == 0) {
        constexpr int kF = FUNC == 1 ? 3 : 1;
        double st[kApx ? 2 * kF : kF];
        st[0] = ve;
        if (FUNC == 1) {
          st[1] = fe.fine;
          st[2] = fe.coarse;
        }
        if (kApx) {
          st[kF] = double(vs);
          if (FUNC == 1) {
            st[kF + 1] = fs.fine;
            st[kF + 2] = fs.coarse;
          }
        }
        regroup(n / kRegroupEvery + bid, sid, st);
        ve = st[0];
        if (FUNC == 1) {
          fe.fine = st[1];
          fe.coarse = st[2];
        }
        if (kApx) {
          vs = float(st[kF]);
          if (FUNC == 1) {
            fs.fine = st[kF + 1];
            fs.coarse = st[kF + 2];
          }
        }
        P = a.path_offset + base + sid;
        plo = uint32_t(P);
        phi = uint32_t(P >> 32);
        cact = base + sid < a.n_paths;
      }
      double u53 = 0.5;
      float u24 = 0.5f;
      if (KIND == AICDF_KIND_APPROX) {
        if ((n & 3u) == 0) w = philox4x32_10(n >> 2, plo, phi, a.tag, a.k0, a.k1);
        u24 = u24_from_word(w[n & 3u]);
      } else {
        if ((n & 1u) == 0) w = philox4x32_10(n >> 1, plo, phi, a.tag, a.k0, a.k1);
        const uint32_t hi = (n & 1u) ? w[2] : w[0], lo = (n & 1u) ? w[3] : w[1];
        u53 = u53_from_words(hi, lo);
        u24 = u24_from_word(hi);
      }
      // approximate step first: in CORRECTION its value, moved to the exact
      // path's lambda, starts the exact inverse's root iteration
      double x0 = 0.0;
      if (kSurr) {
        const float lam = vs * a.lamf;
        // g in [-1, 1] on the trained log-lambda range; outside it the
        // network is evaluated at the range's nearer end (counted; lambda = 0
        // gives -inf).  Hardware log2 and square root (about 1 ulp): the
        // correctly rounded library forms cost ~20 more instructions a step.
        const float gr = fmaf(__builtin_amdgcn_logf(lam), a.g_a, a.g_b);
        const float g = __builtin_amdgcn_fmed3f(gr, -1.0f, 1.0f);
        // all lanes; one path per wavefront: one sample spread over the wave
        const float Pt = SPARSE ? mlp_wave_forward_one(L, xch[threadIdx.x / 64], w2s, dyadic_w16(u24, tab), g)
                                : mlp_wave_forward(L, A, dyadic_w16(u24, tab), g);
        const float s = lam + a.nuf;
        const float x = fmaxf(fmaf(2.0f * __builtin_amdgcn_sqrtf(s), Pt, s), 0.0f);
        fb += (cact && !(gr >= -1.0f && gr <= 1.0f)) ? 1 : 0;
        if (kExact) x0 = double(x) + (ve * a.decay / a.c - double(lam));
        vs = a.cf * x;
        if (FUNC == 1) fs.node(n + 1, N, double(vs));
      }
      if (kPoly) {
        const float lam = vs * a.lamf;
        vs = a.cf * fmaxf(chi2_approx_x<APX>(u24, lam, ctab, a.geo), 0.0f);
        if (kExact) x0 = double(chi2_approx_x<APX>(u24, float(ve * a.decay / a.c), ctab, a.geo));
        if (FUNC == 1) fs.node(n + 1, N, double(vs));
      }
      if (kSank) {
        const float lam = vs * a.lamf;
        vs = a.cf * sankaran_x(u24, lam, a.nuf);
        if (kExact) x0 = double(sankaran_x(u24, float(ve * a.decay / a.c), a.nuf));
        if (FUNC == 1) fs.node(n + 1, N, double(vs));
      }
      if (kEm) {
        const float z = float(exact_phi_inv(double(u24)));
        vs = fmaf(a.xi_sqdt * sqrtf(fabsf(vs)), z, fmaf(a.kdt, a.theta - vs, vs));
        if (FUNC == 1) fs.node(n + 1, N, double(vs));
      }
      if (kExact && work) {
        const double lam = ve * a.decay / a.c;
        // from lambda = 32 on the solver's own start (Sankaran's
        // approximation, relative error ~1e-3 at 30, ~1e-6 at 1000) beats
        // the approximations' (~1e-2), and it is used instead
        if (lam >= 32.0) x0 = 0.0;
        ve = a.c * exact_inverse<SPARSE, kCall>(u53, a.nu, lam, x0, lga1);
        if (FUNC == 1) fe.node(n + 1, N, ve);
      }
    }
    double Y = 0.0, Pf = 0.0, Pc = 0.0;
    if (KIND == AICDF_KIND_APPROX) {
      fs.template result<FUNC>(a.level, N, double(vs), Pf, Pc);
      Y = Pf - Pc;
    } else if (KIND == KIND_TWOWAY) {
      double q;
      fe.template result<FUNC>(a.level, N, ve, Pf, q);
      fs.template result<FUNC>(a.level, N, double(vs), Pc, q);
      Y = Pf - Pc;
    } else {
      fe.template result<FUNC>(a.level, N, ve, Pf, Pc);
      Y = Pf - Pc;
      if (KIND == AICDF_KIND_CORRECTION) {
        double Qf, Qc;
        fs.template result<FUNC>(a.level, N, double(vs), Qf, Qc);
        Y -= Qf - Qc;
      }
    }
    if (kRegroup && N > kRegroupEvery) regroup_return(sid, Y, Pf, Pc);
    if (act) {
      acc.add(Y, Pf, Pc);
      if (path_out) {
        path_out[3 * i] = Y;
        path_out[3 * i + 1] = Pf;
        path_out[3 * i + 2] = Pc;
      }
    }
  }
  block_reduce_store(acc, partials, bid);
  if (kSurr) {
    S.fbs[threadIdx.x] = fb;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int k = 0; k < kLevelBlock; ++k) t += S.fbs[k];
      if (t) atomicAdd(fallbacks, t);
    }
  }
}

// The surrogate's approximate kind one path per thread, held to three waves
// per SIMD (168 registers: the W2 fragments stay in registers across the
// path loop; reading them from LDS at every call frees 32, not enough for a
// fourth wave without spills in the step loop, measured 3x slower).
template <int FUNC>
__global__ __launch_bounds__(kLevelBlock, 3) void cir_level_kernel_surr(CirArgs a, const float* __restrict__ params,
                                                                       const uint16_t* __restrict__ w2b,
                                                                       const f32x4* __restrict__ wtab,
                                                                       double* __restrict__ partials,
                                                                       double* __restrict__ path_out,
                                                                       unsigned long long* __restrict__ fallbacks) {
  __shared__ CirLds<false> S;
  extern __shared__ f32x4 ctab[];
  cir_level_block<AICDF_KIND_APPROX, FUNC, APX_SURROGATE, false, false>(a, params, w2b, wtab, partials, path_out,
                                                                        fallbacks, blockIdx.x, gridDim.x, S, ctab);
}

template <int KIND, int FUNC, int APX, bool SPARSE>
__global__ __launch_bounds__(kLevelBlock) void cir_level_kernel(CirArgs a, const float* __restrict__ params,
                                                               const uint16_t* __restrict__ w2b,
                                                               const f32x4* __restrict__ wtab,
                                                               double* __restrict__ partials,
                                                               double* __restrict__ path_out,
                                                               unsigned long long* __restrict__ fallbacks) {
  constexpr bool kW2 = SPARSE && KIND != AICDF_KIND_EXACT && APX == APX_SURROGATE;
  __shared__ CirLds<kW2> S;
  extern __shared__ f32x4 ctab[];  // APX_POLY*: the chi-squared table (dynamic LDS)
  cir_level_block<KIND, FUNC, APX, SPARSE, kW2>(a, params, w2b, wtab, partials, path_out, fallbacks, blockIdx.x,
                                                gridDim.x, S, ctab);
}

using LevelKernel = void (*)(CirArgs, const float*, const uint16_t*, const f32x4*, double*, double*,
                            unsigned long long*);

// The launch shape (above) of a level: sets a.sparse and the work-group count.
template <int KIND, int APX>
aicdf_status choose_shape(int func, CirArgs& a, size_t lds, unsigned* grid) {
  const LevelKernel ks = func == 0 ? cir_level_kernel<KIND, 0, APX, true> : cir_level_kernel<KIND, 1, APX, true>;
  bool sparse = false;
  if (KIND != AICDF_KIND_APPROX && a.n_paths < kDenseAlways) {
    sparse = a.n_paths <= kSparseAlways;
    if (!sparse) {
      uint64_t w = 0;
      aicdf_status st = resident_waves(reinterpret_cast<const void*>(ks), lds, &w);
      if (st != AICDF_OK) return st;
      const double lam = std::fmax(a.v0, double(a.theta)) * a.decay / a.c;
      sparse = double(a.n_paths) < double(w) * shape_ratio(lam);
    }
  }
  a.sparse = sparse ? 1u : 0u;
  const uint64_t per_block = sparse ? kLevelBlock / 64 : kLevelBlock;
  const uint64_t need = (a.n_paths + per_block - 1) / per_block;
  *grid = unsigned(need < uint64_t(kMaxLevelBlocks) ? need : kMaxLevelBlocks);
  return AICDF_OK;
}

// Chooses the launch shape, sets a.sparse and the grid, launches.
template <int KIND, int APX>
aicdf_status launch_func(int func, CirArgs a, size_t lds, hipStream_t s, const float* p, const uint16_t* w2,
                         const f32x4* wt, double* part, double* po, unsigned long long* fb, unsigned* grid) {
  const LevelKernel ks = func == 0 ? cir_level_kernel<KIND, 0, APX, true> : cir_level_kernel<KIND, 1, APX, true>;
  LevelKernel kd = func == 0 ? cir_level_kernel<KIND, 0, APX, false> : cir_level_kernel<KIND, 1, APX, false>;
  if (KIND == AICDF_KIND_APPROX && APX == APX_SURROGATE)
    kd = func == 0 ? cir_level_kernel_surr<0> : cir_level_kernel_surr<1>;
  aicdf_status st = choose_shape<KIND, APX>(func, a, lds, grid);
  if (st != AICDF_OK) return st;
  hipLaunchKernelGGL(a.sparse ? ks : kd, dim3(*grid), dim3(kLevelBlock), lds, s, a, p, w2, wt, part, po, fb);
  return AICDF_OK;
}

// The shape of a level of any kind (the exact kind's kernel does not depend
// on the approximation: it is the APX_SURROGATE instance).
template <int APX>
aicdf_status choose_shape_kind(int kind, int func, CirArgs& a, size_t lds, unsigned* grid) {
  if (kind == AICDF_KIND_EXACT) return choose_shape<AICDF_KIND_EXACT, APX_SURROGATE>(func, a, 0, grid);
  if (kind == AICDF_KIND_APPROX) return choose_shape<AICDF_KIND_APPROX, APX>(func, a, lds, grid);
  return choose_shape<AICDF_KIND_CORRECTION, APX>(func, a, lds, grid);
}

// The per-level arguments of one job of a batched call; the rest of CirArgs
// is common to the batch.
struct CirJob {
  double c, decay;
  float cf, decayf, lamf, kdt, xi_sqdt;
  uint32_t level, nsteps, tag, sparse;
  uint64_t n_paths, path_offset;
};

struct CirBatch {
  CirArgs base;
  CirJob job[kMaxJobs];
  uint32_t start[kMaxJobs + 1];
  uint32_t n_jobs;
};
// kernel arguments are limited to 4 KiB (with the pointers that follow)
static_assert(sizeof(CirBatch) + 64 <= 4096, "batched CIR arguments exceed the kernel argument limit");

// KSET 0: EXACT jobs only; 1: APPROX jobs only; 2: EXACT, APPROX and
// CORRECTION jobs.  Each work-group finds its job and runs that job's level
// code on its share of the job's paths; fallbacks: one counter per job.
template <int KSET, int FUNC, int APX, bool kW2>
__device__ __forceinline__ void cir_levels_body(const CirBatch& b, const float* __restrict__ params,
                                                const uint16_t* __restrict__ w2b, const f32x4* __restrict__ wtab,
                                                double* __restrict__ partials,
                                                unsigned long long* __restrict__ fallbacks, CirLds<kW2>& S,
                                                f32x4* __restrict__ ctab) {
  uint32_t j = 0;
  while (j + 1 < b.n_jobs && blockIdx.x >= b.start[j + 1]) ++j;
  CirArgs a = b.base;
  const CirJob& jb = b.job[j];
  a.c = jb.c;
  a.decay = jb.decay;
  a.cf = jb.cf;
  a.decayf = jb.decayf;
  a.lamf = jb.lamf;
  a.kdt = jb.kdt;
  a.xi_sqdt = jb.xi_sqdt;
  a.level = jb.level;
  a.nsteps = jb.nsteps;
  a.tag = jb.tag;
  a.sparse = jb.sparse;
  a.n_paths = jb.n_paths;
  a.path_offset = jb.path_offset;
  const uint32_t bid = blockIdx.x - b.start[j], nblk = b.start[j + 1] - b.start[j];
  double* part = partials + size_t(b.start[j]) * kSums;
  unsigned long long* fb = fallbacks + j;
  const int kind = int(a.tag >> 8) - 4;
  if constexpr (KSET == 0) {
    if (a.sparse)
      cir_level_block<AICDF_KIND_EXACT, FUNC, APX, true, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid, nblk, S,
                                                              ctab);
    else
      cir_level_block<AICDF_KIND_EXACT, FUNC, APX, false, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid, nblk,
                                                               S, ctab);
  } else {
    if (KSET == 1 || kind == AICDF_KIND_APPROX) {
      // the approximate kind always runs one path per thread
      cir_level_block<AICDF_KIND_APPROX, FUNC, APX, false, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid, nblk,
                                                                S, ctab);
    } else if constexpr (KSET == 2) {
      if (kind == AICDF_KIND_CORRECTION) {
        if (a.sparse)
          cir_level_block<AICDF_KIND_CORRECTION, FUNC, APX, true, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid,
                                                                       nblk, S, ctab);
        else
          cir_level_block<AICDF_KIND_CORRECTION, FUNC, APX, false, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid,
                                                                        nblk, S, ctab);
      } else {
        if (a.sparse)
          cir_level_block<AICDF_KIND_EXACT, FUNC, APX, true, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid, nblk,
                                                                  S, ctab);
        else
          cir_level_block<AICDF_KIND_EXACT, FUNC, APX, false, kW2>(a, params, w2b, wtab, part, nullptr, fb, bid,
                                                                   nblk, S, ctab);
      }
    }
  }
}

template <int KSET, int FUNC, int APX>
__global__ __launch_bounds__(kLevelBlock) void cir_levels_kernel(CirBatch b, const float* __restrict__ params,
                                                                const uint16_t* __restrict__ w2b,
                                                                const f32x4* __restrict__ wtab,
                                                                double* __restrict__ partials,
                                                                unsigned long long* __restrict__ fallbacks) {
  constexpr bool kW2 = KSET != 0 && APX == APX_SURROGATE;
  __shared__ CirLds<kW2> S;
  extern __shared__ f32x4 ctab[];
  cir_levels_body<KSET, FUNC, APX, kW2>(b, params, w2b, wtab, partials, fallbacks, S, ctab);
}

// APPROX-only batches with the surrogate: three waves per SIMD, as
// cir_level_kernel_surr.
template <int FUNC>
__global__ __launch_bounds__(kLevelBlock, 3) void cir_levels_kernel_surr(CirBatch b, const float* __restrict__ params,
                                                                        const uint16_t* __restrict__ w2b,
                                                                        const f32x4* __restrict__ wtab,
                                                                        double* __restrict__ partials,
                                                                        unsigned long long* __restrict__ fallbacks) {
  __shared__ CirLds<false> S;
  extern __shared__ f32x4 ctab[];
  cir_levels_body<1, FUNC, APX_SURROGATE, false>(b, params, w2b, wtab, partials, fallbacks, S, ctab);
}

template <int KSET, int APX>
void launch_cir_batch(int func, const CirBatch& b, unsigned grid, size_t lds, hipStream_t s, const float* p,
                      const uint16_t* w2, const f32x4* wt, double* part, unsigned long long* fb) {
  if (KSET == 1 && APX == APX_SURROGATE) {
    if (func == 0)
      hipLaunchKernelGGL(cir_levels_kernel_surr<0>, dim3(grid), dim3(kLevelBlock), lds, s, b, p, w2, wt, part, fb);
    else
      hipLaunchKernelGGL(cir_levels_kernel_surr<1>, dim3(grid), dim3(kLevelBlock), lds, s, b, p, w2, wt, part, fb);
    return;
  }
  if (func == 0)
    hipLaunchKernelGGL((cir_levels_kernel<KSET, 0, APX>), dim3(grid), dim3(kLevelBlock), lds, s, b, p, w2, wt, part,
                       fb);
  else
    hipLaunchKernelGGL((cir_levels_kernel<KSET, 1, APX>), dim3(grid), dim3(kLevelBlock), lds, s, b, p, w2, wt, part,
                       fb);
}

template <int APX>
void launch_cir_batch_kset(int kset, int func, const CirBatch& b, unsigned grid, size_t lds, hipStream_t s,
                           const float* p, const uint16_t* w2, const f32x4* wt, double* part, unsigned long long* fb) {
  if (kset == 0)
    launch_cir_batch<0, APX_SURROGATE>(func, b, grid, 0, s, p, w2, wt, part, fb);
  else if (kset == 1)
    launch_cir_batch<1, APX>(func, b, grid, lds, s, p, w2, wt, part, fb);
  else
    launch_cir_batch<2, APX>(func, b, grid, lds, s, p, w2, wt, part, fb);
}

template <int APX>
aicdf_status launch_kind(int kind, int func, const CirArgs& a, size_t lds, hipStream_t s, const float* p,
                         const uint16_t* w2, const f32x4* wt, double* part, double* po, unsigned long long* fb,
                         unsigned* grid) {
  if (kind == AICDF_KIND_EXACT)
    return launch_func<AICDF_KIND_EXACT, APX_SURROGATE>(func, a, 0, s, p, w2, wt, part, po, fb, grid);
  if (kind == AICDF_KIND_APPROX)
    return launch_func<AICDF_KIND_APPROX, APX>(func, a, lds, s, p, w2, wt, part, po, fb, grid);
  if (kind == AICDF_KIND_CORRECTION)
    return launch_func<AICDF_KIND_CORRECTION, APX>(func, a, lds, s, p, w2, wt, part, po, fb, grid);
  return launch_func<KIND_TWOWAY, APX>(func, a, lds, s, p, w2, wt, part, po, fb, grid);
}

// Checks shared by both approximations; fills the common arguments.
aicdf_status cir_setup(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind, uint64_t seed,
                       uint64_t path_offset, const LevelOut& out, CirArgs& a) {
  if (!prm) return fail(AICDF_EINVAL, "params must be non-NULL");
  aicdf_status st = check_level_out(out);
  if (st != AICDF_OK) return st;
  if (level > 12) return fail(AICDF_ERANGE, "level %u > 12", level);
  if (kind < 0 || kind > 3) return fail(AICDF_EINVAL, "kind must be 0, 1, 2 or 3");
  if (prm->functional < 0 || prm->functional > 1 || prm->reserved != 0)
    return fail(AICDF_EINVAL, "functional must be 0 or 1 and reserved 0");
  if (!(prm->kappa > 0.0) || !(prm->theta > 0.0) || !(prm->xi > 0.0) || !(prm->T > 0.0) || !(prm->v0 >= 0.0))
    return fail(AICDF_EINVAL, "need kappa, theta, xi, T > 0 and v0 >= 0");
  if (n_paths > (uint64_t(1) << 40)) return fail(AICDF_ERANGE, "n_paths > 2^40");
  if (path_offset + n_paths < path_offset) return fail(AICDF_ERANGE, "path_offset + n_paths overflows");
  const double nu = 4.0 * prm->kappa * prm->theta / (prm->xi * prm->xi);
  const uint32_t N = 1u << level;
  const double dt = prm->T / N;
  a = CirArgs{};
  a.nu = nu;
  a.decay = std::exp(-prm->kappa * dt);
  a.c = prm->xi * prm->xi * (1.0 - a.decay) / (4.0 * prm->kappa);
  a.v0 = prm->v0;
  a.nuf = float(nu);
  a.cf = float(a.c);
  a.decayf = float(a.decay);
  a.lamf = float(a.decay / a.c);
  a.v0f = float(prm->v0);
  a.level = level;
  a.nsteps = N;
  a.n_paths = n_paths;
  a.path_offset = path_offset;
  a.k0 = uint32_t(seed);
  a.k1 = uint32_t(seed >> 32);
  a.tag = level | (uint32_t(4 + kind) << 8);
  a.kdt = float(prm->kappa * dt);
  a.theta = float(prm->theta);
  a.xi_sqdt = float(prm->xi * std::sqrt(dt));
  return AICDF_OK;
}

// g = 2 (log lambda - lo) / (hi - lo) - 1 as g_a log2(lambda) + g_b.
void surrogate_feature(bool have, double lo, double hi, CirArgs& a) {
  a.g_a = have ? float(2.0 * std::log(2.0) / (hi - lo)) : 0.0f;
  a.g_b = have ? float(-2.0 * lo / (hi - lo) - 1.0) : 0.0f;
}

aicdf_status cir_level_surrogate(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                                 const aicdf_surrogate* sur, uint64_t seed, uint64_t path_offset, const LevelOut& out,
                                 double* path_out, void* stream) {
  CirArgs a;
  unsigned grid = 0;
  aicdf_status st = cir_setup(prm, level, n_paths, kind, seed, path_offset, out, a);
  if (st != AICDF_OK) return st;
  if (kind != AICDF_KIND_EXACT && !sur) return fail(AICDF_EINVAL, "the approximate kinds need a surrogate");
  if (n_paths == 0) return empty_level(static_cast<hipStream_t>(stream), out);
  double snu = a.nu, lo = 0.0, hi = 0.0;
  int sdev = 0, dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  if (sur) {
    surrogate_range(sur, &snu, &lo, &hi, &sdev);
    if (kind != AICDF_KIND_EXACT) {
      if (sdev != dev) return fail(AICDF_EINVAL, "surrogate lives on device %d, current device is %d", sdev, dev);
      if (std::fabs(snu - a.nu) > 1e-12 * a.nu)
        return fail(AICDF_EINVAL, "surrogate was built for nu = %.17g, the process has nu = %.17g", snu, a.nu);
    }
  }
  surrogate_feature(sur != nullptr, lo, hi, a);

  auto s = static_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  const float* p = sur ? surrogate_params(sur) : nullptr;
  const uint16_t* w2 = sur ? surrogate_w2b(sur) : nullptr;
  const f32x4* wt = sur ? reinterpret_cast<const f32x4*>(surrogate_wtab(sur)) : nullptr;
  st = begin_level(ws, s, out);
  if (st != AICDF_OK) return st;
  st = launch_kind<APX_SURROGATE>(kind, prm->functional, a, 0, s, p, w2, wt, ws->partials, path_out, ws->counter,
                                  &grid);
  if (st != AICDF_OK) return st;
  AICDF_HIP(hipGetLastError());
  return finish_level(ws, grid, s, double(n_paths), out);
}

aicdf_status cir_level_table(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                             const aicdf_chi2_table* tab, uint64_t seed, uint64_t path_offset, const LevelOut& out,
                             double* path_out, void* stream) {
  CirArgs a;
  unsigned grid = 0;
  aicdf_status st = cir_setup(prm, level, n_paths, kind, seed, path_offset, out, a);
  if (st != AICDF_OK) return st;
  if (kind != AICDF_KIND_EXACT && !tab) return fail(AICDF_EINVAL, "the approximate kinds need a table");
  if (n_paths == 0) return empty_level(static_cast<hipStream_t>(stream), out);
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  Chi2Info ti{};
  size_t lds = 0;
  if (tab && kind != AICDF_KIND_EXACT) {
    ti = chi2_info(tab);
    if (ti.device != dev) return fail(AICDF_EINVAL, "table lives on device %d, current device is %d", ti.device, dev);
    if (std::fabs(ti.nu - a.nu) > 1e-12 * a.nu)
      return fail(AICDF_EINVAL, "table was built for nu = %.17g, the process has nu = %.17g", ti.nu, a.nu);
    a.geo = Chi2Geom{float(ti.nu), float(std::sqrt(ti.nu)), float(ti.n_knots - 1), ti.n_knots - 2, ti.n_intervals};
    a.table_rows = ti.n_knots * 2 * ti.n_intervals;
    if (a.table_rows > kMaxLdsRows)
      return fail(AICDF_EINVAL, "table has %u rows; the CIR level stages at most %u in LDS", a.table_rows,
                  kMaxLdsRows);
    lds = size_t(a.table_rows) * sizeof(f32x4);
  }

  auto s = static_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  const auto* wt = static_cast<const f32x4*>(ti.dev_rows);
  st = begin_level(ws, s, out);
  if (st != AICDF_OK) return st;
  if (kind == AICDF_KIND_EXACT || ti.degree == 1)
    st = launch_kind<APX_POLY1>(kind, prm->functional, a, lds, s, nullptr, nullptr, wt, ws->partials, path_out,
                                ws->counter, &grid);
  else
    st = launch_kind<APX_POLY3>(kind, prm->functional, a, lds, s, nullptr, nullptr, wt, ws->partials, path_out,
                                ws->counter, &grid);
  if (st != AICDF_OK) return st;
  AICDF_HIP(hipGetLastError());
  return finish_level(ws, grid, s, double(n_paths), out);
}

aicdf_status cir_level_em(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                          uint64_t seed, uint64_t path_offset, const LevelOut& out, double* path_out, void* stream) {
  CirArgs a;
  unsigned grid = 0;
  aicdf_status st = cir_setup(prm, level, n_paths, kind, seed, path_offset, out, a);
  if (st != AICDF_OK) return st;
  if (n_paths == 0) return empty_level(static_cast<hipStream_t>(stream), out);
  auto s = static_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  st = begin_level(ws, s, out);
  if (st != AICDF_OK) return st;
  st = launch_kind<APX_EM>(kind, prm->functional, a, 0, s, nullptr, nullptr, nullptr, ws->partials, path_out,
                           ws->counter, &grid);
  if (st != AICDF_OK) return st;
  AICDF_HIP(hipGetLastError());
  return finish_level(ws, grid, s, double(n_paths), out);
}

aicdf_status cir_level_sankaran(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                                uint64_t seed, uint64_t path_offset, const LevelOut& out, double* path_out,
                                void* stream) {
  CirArgs a;
  unsigned grid = 0;
  aicdf_status st = cir_setup(prm, level, n_paths, kind, seed, path_offset, out, a);
  if (st != AICDF_OK) return st;
  if (n_paths == 0) return empty_level(static_cast<hipStream_t>(stream), out);
  auto s = static_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  st = begin_level(ws, s, out);
  if (st != AICDF_OK) return st;
  st = launch_kind<APX_SANKARAN>(kind, prm->functional, a, 0, s, nullptr, nullptr, nullptr, ws->partials,
                                 path_out, ws->counter, &grid);
  if (st != AICDF_OK) return st;
  AICDF_HIP(hipGetLastError());
  return finish_level(ws, grid, s, double(n_paths), out);
}

template <int APX>
aicdf_status cir_batch_apx(const aicdf_cir_params* prm, const aicdf_level_job* jobs, uint32_t n_jobs,
                           const CirArgs& common, size_t lds, uint64_t seed, double* sums_dev, hipStream_t s,
                           const float* p, const uint16_t* w2, const f32x4* wt) {
  CirBatch b{};
  JobSpans sp{};
  b.n_jobs = sp.n_jobs = n_jobs;
  bool any_exact = false, any_approx = false, any_corr = false;
  uint32_t total = 0;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    const aicdf_level_job& jb = jobs[j];
    CirArgs a;
    aicdf_status st = cir_setup(prm, jb.level, jb.n_paths, jb.kind, seed, jb.path_offset,
                                LevelOut{nullptr, sums_dev}, a);
    if (st == AICDF_OK && jb.kind == KIND_TWOWAY) st = fail(AICDF_EINVAL, "the two-way kind is not batched");
    unsigned g = 0;
    if (st == AICDF_OK && jb.n_paths > 0) {
      a.g_a = common.g_a;
      a.g_b = common.g_b;
      a.geo = common.geo;
      a.table_rows = common.table_rows;
      st = choose_shape_kind<APX>(jb.kind, prm->functional, a, lds, &g);
    }
    if (st != AICDF_OK) {
      const std::string msg = aicdf_last_error();
      return fail(st, "job %u: %s", j, msg.c_str());
    }
    if (j == 0) {
      b.base = a;
      b.base.g_a = common.g_a;
      b.base.g_b = common.g_b;
      b.base.geo = common.geo;
      b.base.table_rows = common.table_rows;
    }
    b.job[j] = CirJob{a.c, a.decay, a.cf, a.decayf, a.lamf, a.kdt, a.xi_sqdt, a.level, a.nsteps, a.tag, a.sparse,
                      a.n_paths, a.path_offset};
    any_exact |= jb.kind == AICDF_KIND_EXACT;
    any_approx |= jb.kind == AICDF_KIND_APPROX;
    any_corr |= jb.kind == AICDF_KIND_CORRECTION;
    sp.start[j] = b.start[j] = total;
    sp.n_paths[j] = double(jb.n_paths);
    total += g;
  }
  sp.start[n_jobs] = b.start[n_jobs] = total;
  Workspace* ws = nullptr;
  aicdf_status st = get_workspace(s, &ws);
  if (st != AICDF_OK) return st;
  std::lock_guard<std::mutex> lock(ws->mu);
  st = get_batch_buffers(ws);
  if (st != AICDF_OK) return st;
  if (total > 0) {
    const int kset = (!any_approx && !any_corr) ? 0 : (!any_exact && !any_corr) ? 1 : 2;
    launch_cir_batch_kset<APX>(kset, prm->functional, b, total, lds, s, p, w2, wt, ws->batch_partials,
                               ws->batch_counters);
    AICDF_HIP(hipGetLastError());
  }
  return reduce_batch(ws->batch_partials, sp, ws->batch_counters, sums_dev, s);
}

aicdf_status cir_batch(const aicdf_cir_params* prm, const aicdf_level_job* jobs, uint32_t n_jobs, int32_t apx,
                       const void* approx, uint64_t seed, double* sums_dev, void* stream) {
  if (!prm) return fail(AICDF_EINVAL, "params must be non-NULL");
  if (n_jobs == 0) return ok();
  if (!jobs || !sums_dev) return fail(AICDF_EINVAL, "jobs and sums_dev must be non-NULL");
  if (n_jobs > uint32_t(kMaxJobs)) return fail(AICDF_ERANGE, "%u jobs > %d", n_jobs, kMaxJobs);
  if (reinterpret_cast<uintptr_t>(sums_dev) & 7u) return fail(AICDF_EINVAL, "sums_dev must be 8-byte aligned");
  if (apx < AICDF_CIR_SURROGATE || apx > AICDF_CIR_SANKARAN) return fail(AICDF_EINVAL, "unknown approximation %d", apx);
  bool any_apx = false;
  for (uint32_t j = 0; j < n_jobs; ++j) any_apx |= jobs[j].kind != AICDF_KIND_EXACT;
  if (any_apx && !approx && (apx == AICDF_CIR_SURROGATE || apx == AICDF_CIR_TABLE))
    return fail(AICDF_EINVAL, "the approximate kinds need a surrogate or table");
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  const double nu = 4.0 * prm->kappa * prm->theta / (prm->xi * prm->xi);
  auto s = static_cast<hipStream_t>(stream);
  CirArgs common{};
  if (apx == AICDF_CIR_SURROGATE) {
    const auto* sur = static_cast<const aicdf_surrogate*>(approx);
    double snu = nu, lo = 0.0, hi = 0.0;
    int sdev = dev;
    if (sur) {
      surrogate_range(sur, &snu, &lo, &hi, &sdev);
      if (any_apx && sdev != dev)
        return fail(AICDF_EINVAL, "surrogate lives on device %d, current device is %d", sdev, dev);
      if (any_apx && std::fabs(snu - nu) > 1e-12 * nu)
        return fail(AICDF_EINVAL, "surrogate was built for nu = %.17g, the process has nu = %.17g", snu, nu);
    }
    surrogate_feature(sur != nullptr, lo, hi, common);
    const float* p = sur ? surrogate_params(sur) : nullptr;
    const uint16_t* w2 = sur ? surrogate_w2b(sur) : nullptr;
    const f32x4* wt = sur ? reinterpret_cast<const f32x4*>(surrogate_wtab(sur)) : nullptr;
    return cir_batch_apx<APX_SURROGATE>(prm, jobs, n_jobs, common, 0, seed, sums_dev, s, p, w2, wt);
  }
  if (apx == AICDF_CIR_TABLE) {
    const auto* tab = static_cast<const aicdf_chi2_table*>(approx);
    Chi2Info ti{};
    size_t lds = 0;
    if (tab) {
      ti = chi2_info(tab);
      if (any_apx && ti.device != dev)
        return fail(AICDF_EINVAL, "table lives on device %d, current device is %d", ti.device, dev);
      if (any_apx && std::fabs(ti.nu - nu) > 1e-12 * nu)
        return fail(AICDF_EINVAL, "table was built for nu = %.17g, the process has nu = %.17g", ti.nu, nu);
      common.geo = Chi2Geom{float(ti.nu), float(std::sqrt(ti.nu)), float(ti.n_knots - 1), ti.n_knots - 2,
                            ti.n_intervals};
      common.table_rows = ti.n_knots * 2 * ti.n_intervals;
      if (common.table_rows > kMaxLdsRows)
        return fail(AICDF_EINVAL, "table has %u rows; the CIR level stages at most %u in LDS", common.table_rows,
                    kMaxLdsRows);
      lds = size_t(common.table_rows) * sizeof(f32x4);
    }
    const auto* wt = static_cast<const f32x4*>(ti.dev_rows);
    if (!tab || ti.degree == 1)
      return cir_batch_apx<APX_POLY1>(prm, jobs, n_jobs, common, lds, seed, sums_dev, s, nullptr, nullptr, wt);
    return cir_batch_apx<APX_POLY3>(prm, jobs, n_jobs, common, lds, seed, sums_dev, s, nullptr, nullptr, wt);
  }
  if (apx == AICDF_CIR_EM)
    return cir_batch_apx<APX_EM>(prm, jobs, n_jobs, common, 0, seed, sums_dev, s, nullptr, nullptr, nullptr);
  return cir_batch_apx<APX_SANKARAN>(prm, jobs, n_jobs, common, 0, seed, sums_dev, s, nullptr, nullptr, nullptr);
}

}  // namespace

extern "C" aicdf_status mlmc_levels_cir(const aicdf_cir_params* prm, const aicdf_level_job* jobs, uint32_t n_jobs,
                                        int32_t approx_type, const void* approx, uint64_t seed, double* sums_dev,
                                        void* stream) {
  return cir_batch(prm, jobs, n_jobs, approx_type, approx, seed, sums_dev, stream);
}

extern "C" aicdf_status mlmc_level_cir(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                                       const aicdf_surrogate* sur, uint64_t seed, uint64_t path_offset,
                                       aicdf_level_sums* out, double* path_out, void* stream) {
  if (!out) return fail(AICDF_EINVAL, "out must be non-NULL");
  return cir_level_surrogate(prm, level, n_paths, kind, sur, seed, path_offset, LevelOut{out, nullptr}, path_out,
                             stream);
}

extern "C" aicdf_status mlmc_level_cir_table(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths,
                                             int32_t kind, const aicdf_chi2_table* tab, uint64_t seed,
                                             uint64_t path_offset, aicdf_level_sums* out, double* path_out,
                                             void* stream) {
  if (!out) return fail(AICDF_EINVAL, "out must be non-NULL");
  return cir_level_table(prm, level, n_paths, kind, tab, seed, path_offset, LevelOut{out, nullptr}, path_out, stream);
}

extern "C" aicdf_status mlmc_level_cir_em(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths, int32_t kind,
                                          uint64_t seed, uint64_t path_offset, aicdf_level_sums* out,
                                          double* path_out, void* stream) {
  if (!out) return fail(AICDF_EINVAL, "out must be non-NULL");
  return cir_level_em(prm, level, n_paths, kind, seed, path_offset, LevelOut{out, nullptr}, path_out, stream);
}

extern "C" aicdf_status mlmc_level_cir_sankaran(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths,
                                                int32_t kind, uint64_t seed, uint64_t path_offset,
                                                aicdf_level_sums* out, double* path_out, void* stream) {
  if (!out) return fail(AICDF_EINVAL, "out must be non-NULL");
  return cir_level_sankaran(prm, level, n_paths, kind, seed, path_offset, LevelOut{out, nullptr}, path_out, stream);
}

extern "C" aicdf_status mlmc_level_cir_async(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths,
                                             int32_t kind, const aicdf_surrogate* sur, uint64_t seed,
                                             uint64_t path_offset, double* sums_dev, double* path_out, void* stream) {
  if (!sums_dev) return fail(AICDF_EINVAL, "sums_dev must be non-NULL");
  return cir_level_surrogate(prm, level, n_paths, kind, sur, seed, path_offset, LevelOut{nullptr, sums_dev},
                             path_out, stream);
}

extern "C" aicdf_status mlmc_level_cir_table_async(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths,
                                                   int32_t kind, const aicdf_chi2_table* tab, uint64_t seed,
                                                   uint64_t path_offset, double* sums_dev, double* path_out,
                                                   void* stream) {
  if (!sums_dev) return fail(AICDF_EINVAL, "sums_dev must be non-NULL");
  return cir_level_table(prm, level, n_paths, kind, tab, seed, path_offset, LevelOut{nullptr, sums_dev}, path_out,
                         stream);
}

extern "C" aicdf_status mlmc_level_cir_em_async(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths,
                                                int32_t kind, uint64_t seed, uint64_t path_offset, double* sums_dev,
                                                double* path_out, void* stream) {
  if (!sums_dev) return fail(AICDF_EINVAL, "sums_dev must be non-NULL");
  return cir_level_em(prm, level, n_paths, kind, seed, path_offset, LevelOut{nullptr, sums_dev}, path_out, stream);
}

extern "C" aicdf_status mlmc_level_cir_sankaran_async(const aicdf_cir_params* prm, uint32_t level, uint64_t n_paths,
                                                      int32_t kind, uint64_t seed, uint64_t path_offset,
                                                      double* sums_dev, double* path_out, void* stream) {
  if (!sums_dev) return fail(AICDF_EINVAL, "sums_dev must be non-NULL");
  return cir_level_sankaran(prm, level, n_paths, kind, seed, path_offset, LevelOut{nullptr, sums_dev}, path_out,
                            stream);
}
