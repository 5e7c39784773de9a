// The learned surrogate of Section 5.1's rescaled inverse non-central
// chi-squared CDF: parameters, batched inference, training (forward and
// backward on the BF16 matrix cores, FP32 master weights, Adam), the exact
// FP64 training targets, and persistence.
//
// Training, per work-group of one wave (64 samples):
//   forward   as mlp_wave_forward (mlp_device.hpp), keeping bf16(h1), a2;
//   output    r = P~ - P, dP = 2 r / batch (mean squared error);
//   layer 3   dW3[m] = sum_s dP_s h2[s][m], db3 = sum_s dP_s;
//   layer 2   da2 = dP W3 relu'(a2); db2 = sum_s da2;
//             dW2 = da2^T bf16(h1)      on MFMA (M = out, N = in, K = sample)
//             dH1^T = bf16(W2)^T da2^T  on MFMA (M = in, N = sample, K = out)
//             (da2 enters both products rounded to BF16; the rounding of h1
//             and W2 is passed straight through)
//   layer 1   da1 = dH1 relu'(a1), dW1 = sum_s da1 [w, g], db1 = sum_s da1.
// Operands are transposed through LDS.  Every work-group writes its partial
// gradient (4417 floats); two passes sum the partials in a fixed order
// (slices of blocks, then the slices) and apply Adam, so training is
// deterministic for a given seed.
#include <cmath>
#include <cstring>
#include <fstream>

#include "internal.hpp"
#include "mlp_device.hpp"
#include "ncx2_device.hpp"

using namespace aicdf;

struct aicdf_surrogate {
  double nu, lo, hi;
  int device;
  float* params;     // device, kNParams FP32 master
  uint16_t* w2b;     // device, 64 x 64 BF16 copy of W2
  uint16_t* w2bt;    // device, its transpose in the training kernel's K-slot order
  float* adam_m;     // device
  float* adam_v;     // device
  float* wtab;       // device, 64 rows x 4 floats: cubic dyadic table for w
  float* partials;   // device, max_blocks x kNParams
  float* loss_part;  // device, max_blocks
  double* scratch;   // device, kNParams + 1 doubles (reduced gradient, loss)
  double* stage;     // device, kMaxSlices x (kNParams + 1): sums of block slices
  size_t max_blocks;
  uint64_t step;
};

namespace {

constexpr int kTrainWave = 64;
// version 2: relu activations (version 1 files hold weights of another network)
constexpr uint32_t kFileVersion = 2;
constexpr size_t kMaxTrainBlocks = 4096;  // 262144 samples per call of the train kernel
// the per-block partial gradients are summed in two fixed-order stages: up to
// kMaxSlices slices of at least kSliceRows blocks each, then the slices
constexpr unsigned kMaxSlices = 32, kSliceRows = 32;

// w = D(u): the 16-row cubic dyadic approximation in FP32 (Algorithm 1), rows
// zero-padded to four coefficients.
__device__ __forceinline__ float dyadic_w(float u, const f32x4* __restrict__ tab) {
  const bool p = u < 0.5f;
  const float ur = p ? u : 1.0f - u;
  const uint32_t e = min(126u - (__float_as_uint(ur) >> 23), 15u);
  const float s = ur * __uint_as_float((128u + e) << 23);
  const f32x4 c = tab[e];
  const float z = fmaf(fmaf(fmaf(c[3], s, c[2]), s, c[1]), s, c[0]);
  return p ? z : -z;
}

// ---------------------------------------------------------------- inference
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ params,
                                                          const uint16_t* __restrict__ w2b,
                                                          const f32x4* __restrict__ wtab, size_t n,
                                                          const float* __restrict__ u,
                                                          const float* __restrict__ loglam, float* __restrict__ p,
                                                          float lo, float inv_span2) {
  __shared__ MlpLds L;
  __shared__ f32x4 tab[16];
  mlp_stage_params(L, params, threadIdx.x, 256);
  if (threadIdx.x < 16) tab[threadIdx.x] = wtab[threadIdx.x];
  __syncthreads();
  bf16x8 A[2][4];
  mlp_load_w2(w2b, A);
  const size_t wave = threadIdx.x >> 6;
  for (size_t base = (size_t(blockIdx.x) * 4 + wave) * 64; base < n; base += size_t(gridDim.x) * 256) {
    const size_t i = base + __lane_id();
    const bool act = i < n;
    const float ui = act ? u[i] : 0.5f;
    const float gi = act ? mlp_g(loglam[i], lo, inv_span2) : 0.0f;
    const float out = mlp_wave_forward(L, A, dyadic_w(ui, tab), gi);
    if (act) p[i] = out;
  }
}

// ---------------------------------------------------------------- training
// K slot k of the dH1 product holds output unit swap23(k) (bits 2 and 3 of k
// exchanged): slot 16 kt + 8 h + i is then unit mlp_unit(kt / 2, 8 (kt % 2) +
// i, h), the unit that a lane of half h holds in its layer-2 result slot
// j = 8 (kt % 2) + i of tile kt / 2, so that each lane's own bf16(da2)
// values are its B fragments and need no transpose.
__host__ __device__ constexpr int swap23(int k) { return (k & ~12) | ((k & 4) << 1) | ((k & 8) >> 1); }

struct TrainLds {
  MlpLds P;
  bf16x8 a1n[2][64];  // layer-1 A fragments with rows in natural unit order (zero in lanes 32..63)
  f32x4 tab[16];
  union {
    struct {
      uint16_t h1t[kHidden * kHidden];     // bf16(h1)  [in][sample]
      uint16_t da2_ms[kHidden * kHidden];  // bf16(da2) [out][sample]
    } t;
    float red[64][33];  // per-unit sums over samples (after the dW2 product)
  } u;
};

__device__ __forceinline__ uint16_t bits(__bf16 x) { return __builtin_bit_cast(uint16_t, x); }

// Sum over the 32 lanes of each half of a per-lane vector of 32 values;
// lane l returns the total of slot (l & 31) of half (l >> 5).
__device__ __forceinline__ float half_sum(TrainLds& S, const float (&v)[32]) {
  const int l = threadIdx.x;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 32; ++i) S.u.red[l][i] = v[i];
  __syncthreads();
  const int idx = l & 31, h = l >> 5;
  float s = 0.0f;
  for (int rr = 0; rr < 32; ++rr) s += S.u.red[h * 32 + rr][idx];
  return s;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// One work-group of one wave: 64 samples.  w2bt: bf16(W2)^T with its
// columns in K-slot order, w2bt[in][k] = bf16(W2[swap23(k)][in]).  Held to
// 256 registers (two waves per SIMD; the compiler's own choice, 251 + 80
// accumulation registers, leaves one).
__global__ __launch_bounds__(kTrainWave) __attribute__((amdgpu_waves_per_eu(2))) void mlp_train_kernel(
    const float* __restrict__ params, const uint16_t* __restrict__ w2b, const uint16_t* __restrict__ w2bt,
    const f32x4* __restrict__ wtab, const float* __restrict__ u, const float* __restrict__ loglam,
    const float* __restrict__ target, size_t n_data, uint64_t perm_a, uint64_t perm_b, size_t first, size_t count,
    float inv_batch, float lo, float inv_span2, float* __restrict__ partials, float* __restrict__ loss_part) {
  __shared__ TrainLds S;
  const int l = threadIdx.x, r = l & 31, half = l >> 5;
  mlp_stage_params(S.P, params, l, kTrainWave);
  {
    // natural-order rows: row k is hidden unit k
    __bf16 wh, wl, gh, gl, bh, bl;
    split_bf16(params[kOffW1 + 2 * l], wh, wl);
    split_bf16(params[kOffW1 + 2 * l + 1], gh, gl);
    split_bf16(params[kOffB1 + l], bh, bl);
    const __bf16 zero = to_bf16(0.0f);
    S.a1n[l >> 5][l & 31] = bf16x8{wh, wl, wh, gh, gl, gh, bh, bl};
    S.a1n[l >> 5][32 + (l & 31)] = bf16x8{zero, zero, zero, zero, zero, zero, zero, zero};
  }
  if (l < 16) S.tab[l] = wtab[l];
  __syncthreads();

  // ---- sample of this lane (permuted index; lanes past the batch are masked)
  const size_t k = size_t(blockIdx.x) * kTrainWave + l;
  const bool act = k < count;
  float ui = 0.5f, gi = 0.0f, ti = 0.0f;
  if (act) {
    const size_t idx = size_t((perm_a * uint64_t(first + k) + perm_b) % uint64_t(n_data));
    ui = u[idx];
    gi = mlp_g(loglam[idx], lo, inv_span2);
    ti = target[idx];
  }
  const float w = dyadic_w(ui, S.tab);
  if (!act) ti = w;

  // ---- forward: the arithmetic of mlp_wave_forward, keeping bf16(h1), a2
  bf16x8 A[2][4];
  mlp_load_w2(w2b, A);
  const float wo = __shfl_xor(w, 32), go = __shfl_xor(gi, 32);
  const float ws[2] = {half ? wo : w, half ? w : wo};  // inputs of samples r, r + 32
  const float gs[2] = {half ? go : gi, half ? gi : go};
  const bf16x8 X[2] = {mlp_input_frag(w, gi), mlp_input_frag(wo, go)};
  bf16x8 B[2][4];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) mlp_layer1_mfma(mlp_w1_frag(S.P, 0), mlp_w1_frag(S.P, 1), X[nt], B[nt]);
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int i = 0; i < 8; ++i) S.u.t.h1t[(16 * kt + 8 * half + i) * kHidden + 32 * nt + r] = bits(B[nt][kt][i]);
  f32x16 acc[2][2];  // a2 = W2 bf16(h1) + b2, [mt][nt]
  float part[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    float p = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x16 c = mlp_b2_acc(S.P, mt, half);
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mt][kt], B[nt][kt], c, 0, 0, 0);
      acc[mt][nt] = c;
#pragma unroll
      for (int j = 0; j < 16; ++j) p = fmaf(S.P.w3s[mt][half][j], mlp_act(c[j]), p);
    }
    part[nt] = p + __shfl_xor(p, 32);
  }
  const float P = w + (half ? part[1] : part[0]) + S.P.b3;

  // ---- output gradient
  const float res = act ? P - ti : 0.0f;
  const float dP = 2.0f * res * inv_batch;
  const float dPo = __shfl_xor(dP, 32);
  const float dPs[2] = {half ? dPo : dP, half ? dP : dPo};

  // ---- layers 3 and 2 (elementwise part); bf16(da2) as the dH1 B
  // fragments (K slot order swap23) and, transposed, for dW2
  float gW3[32], gb2[32];
  bf16x8 Bd[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int m = mlp_unit(mt, j, half);
      const float w3 = S.P.w3s[mt][half][j];
      float s3 = 0.0f, s2 = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const float a2 = acc[mt][nt][j];
        const float da2 = dPs[nt] * w3 * mlp_act_grad(a2);
        s3 = fmaf(dPs[nt], mlp_act(a2), s3);
        s2 += da2;
        const __bf16 db = to_bf16(da2);
        Bd[nt][2 * mt + (j >> 3)][j & 7] = db;
        S.u.t.da2_ms[m * kHidden + 32 * nt + r] = bits(db);
      }
      gW3[mt * 16 + j] = s3;
      gb2[mt * 16 + j] = s2;
    }
  __syncthreads();

  float* out = partials + size_t(blockIdx.x) * kNParams;
  // ---- dW2 = da2^T bf16(h1): M = out, N = in, K = sample
  {
    bf16x8 Aa[2][4], Bb[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        Aa[t][kt] = *reinterpret_cast<const bf16x8*>(&S.u.t.da2_ms[(32 * t + r) * kHidden + 16 * kt + 8 * half]);
        Bb[t][kt] = *reinterpret_cast<const bf16x8*>(&S.u.t.h1t[(32 * t + r) * kHidden + 16 * kt + 8 * half]);
      }
    f32x16 g2[2][2];
    mlp_layer2(Aa, Bb, g2);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          out[kOffW2 + mlp_unit(mt, j, half) * kHidden + 32 * nt + r] = g2[mt][nt][j];
  }
  // ---- reductions over samples of the per-unit vectors of layers 3 and 2
  // (LDS of the transposes is free from here on)
  const int unit = mlp_unit((l & 31) >> 4, l & 15, half);
  float v;
  v = half_sum(S, gW3);
  out[kOffW3 + unit] = v;
  v = half_sum(S, gb2);
  out[kOffB2 + unit] = v;
  // ---- dH1^T = bf16(W2)^T da2^T: M = in, N = sample, K = out (slot order
  // swap23); then layer 1, with relu'(a1) from the layer-1 product with rows
  // in natural order (the result layout of dH1^T)
  float gw0[32], gw1[32], gb1[32];
  {
    bf16x8 Aw[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        Aw[t][kt] = *reinterpret_cast<const bf16x8*>(w2bt + (32 * t + r) * kHidden + 16 * kt + 8 * half);
    f32x16 dh[2][2];
    mlp_layer2(Aw, Bd, dh);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      float s0[16], s1[16], sb[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) s0[j] = s1[j] = sb[j] = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const f32x16 a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a1n[mt][l], X[nt], f32x16{}, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const float da1 = dh[mt][nt][j] * mlp_act_grad(a1[j]);
          s0[j] = fmaf(da1, ws[nt], s0[j]);
          s1[j] = fmaf(da1, gs[nt], s1[j]);
          sb[j] += da1;
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        gw0[mt * 16 + j] = s0[j];
        gw1[mt * 16 + j] = s1[j];
        gb1[mt * 16 + j] = sb[j];
      }
    }
  }
  // ---- and of layer 1
  v = half_sum(S, gw0);
  out[kOffW1 + 2 * unit] = v;
  v = half_sum(S, gw1);
  out[kOffW1 + 2 * unit + 1] = v;
  v = half_sum(S, gb1);
  out[kOffB1 + unit] = v;
  const float db3 = wave_sum(dP);
  const float ls = wave_sum(res * res);
  if (l == 0) {
    out[kOffB3] = db3;
    loss_part[blockIdx.x] = ls;
  }
}

// First stage: slice blockIdx.y of the per-block partials (blocks
// [y rows, min((y + 1) rows, nblocks))), summed in order in FP64; entry
// kNParams is the loss.
__global__ __launch_bounds__(256) void mlp_slice_sum_kernel(const float* __restrict__ partials,
                                                            const float* __restrict__ loss_part, unsigned nblocks,
                                                            unsigned rows, double* __restrict__ stage) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > kNParams) return;
  const unsigned b0 = blockIdx.y * rows, b1 = min(b0 + rows, nblocks);
  double g = 0.0;
  if (p == kNParams) {
    for (unsigned b = b0; b < b1; ++b) g += loss_part[b];
  } else {
    // unrolled so that the loads are in flight together; the sum keeps its order
#pragma unroll 16
    for (unsigned b = b0; b < b1; ++b) g += partials[size_t(b) * kNParams + p];
  }
  stage[size_t(blockIdx.y) * (kNParams + 1) + p] = g;
}

// Second stage: the sum of the slices (in order) and, for mode 1, one Adam
// step on the FP32 master weights with a refresh of the BF16 W2 copy.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const double* __restrict__ stage, unsigned slices,
                                                         double* __restrict__ grad_out, float* __restrict__ params,
                                                         float* __restrict__ am, float* __restrict__ av,
                                                         uint16_t* __restrict__ w2b, uint16_t* __restrict__ w2bt,
                                                         int adam, float lr, float bc1, float bc2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > kNParams) return;
  double g = 0.0;
#pragma unroll 16
  for (unsigned y = 0; y < slices; ++y) g += stage[size_t(y) * (kNParams + 1) + p];
  if (p == kNParams) {
    grad_out[kNParams] += g;  // running loss sum
    return;
  }
  if (!adam) {
    grad_out[p] = g;
    return;
  }
  const float gf = float(g);
  const float m = 0.9f * am[p] + 0.1f * gf;
  const float v = 0.999f * av[p] + 0.001f * gf * gf;
  am[p] = m;
  av[p] = v;
  const float mh = m / bc1, vh = v / bc2;
  const float np = params[p] - lr * mh / (sqrtf(vh) + 1e-8f);
  params[p] = np;
  if (p >= kOffW2 && p < kOffW2 + kHidden * kHidden) {
    const int q = p - kOffW2, o = q / kHidden, i = q % kHidden;
    w2b[q] = w2bt[i * kHidden + swap23(o)] = f32_to_bf16_bits(np);
  }
}

__global__ __launch_bounds__(256) void w2_refresh_kernel(const float* __restrict__ params, uint16_t* __restrict__ w2b,
                                                         uint16_t* __restrict__ w2bt) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < kHidden * kHidden)
    w2b[q] = w2bt[(q % kHidden) * kHidden + swap23(q / kHidden)] = f32_to_bf16_bits(params[kOffW2 + q]);
}

// ---------------------------------------------------------------- training data
// Sample i: Philox block (i mod 2^32, i / 2^32, 0x5EED, 0) with key seed.
// Word 1 selects the tail-weighted eighth (u = 2^(-24 v), v on the u24 grid,
// mirrored when bit 3 of word 1 is set); otherwise u is the u24 value of word
// 0; log lambda = lo + (hi - lo) u24(word 3).  Target: Section 5.1's P from
// the exact FP64 inverse at lambda = exp(log lambda as stored).
__global__ __launch_bounds__(256) void make_data_kernel(uint32_t k0, uint32_t k1, size_t n, double nu, float lo,
                                                        float hi, float* __restrict__ u, float* __restrict__ loglam,
                                                        float* __restrict__ target) {
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
    const u32x4 wd = philox4x32_10(uint32_t(i), uint32_t(i >> 32), 0x5EEDu, 0u, k0, k1);
    float ui;
    if ((wd[1] & 7u) == 0u) {
      ui = exp2f(-24.0f * u24_from_word(wd[2]));
      if ((wd[1] >> 3) & 1u) ui = 1.0f - ui;
      ui = fminf(fmaxf(ui, 0x1p-24f), 1.0f - 0x1p-24f);
    } else {
      ui = u24_from_word(wd[0]);
    }
    const float ll = fmaf(hi - lo, u24_from_word(wd[3]), lo);
    const double lam = exp(double(ll));
    const double x = ncx2_icdf(double(ui), nu, lam);
    const double s = lam + nu;
    u[i] = ui;
    loglam[i] = ll;
    target[i] = float((x - s) / (2.0 * sqrt(s)));
  }
}

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

aicdf_status check_dev(const aicdf_surrogate* s) {
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  if (dev != s->device) return fail(AICDF_EINVAL, "surrogate lives on device %d, current device is %d", s->device, dev);
  return AICDF_OK;
}

void free_surrogate(aicdf_surrogate* s) {
  if (!s) return;
  for (void* p : {(void*)s->params, (void*)s->w2b, (void*)s->w2bt, (void*)s->adam_m, (void*)s->adam_v, (void*)s->wtab,
                  (void*)s->partials, (void*)s->loss_part, (void*)s->scratch, (void*)s->stage})
    if (p) (void)hipFree(p);
  delete s;
}

aicdf_status alloc_surrogate(double nu, double lo, double hi, aicdf_surrogate** out) {
  auto* s = new (std::nothrow) aicdf_surrogate();
  if (!s) return fail(AICDF_ENOMEM, "host allocation failed");
  std::memset(s, 0, sizeof *s);
  s->nu = nu;
  s->lo = lo;
  s->hi = hi;
  s->max_blocks = kMaxTrainBlocks;
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipMalloc(&s->params, kNParams * 4) != hipSuccess || hipMalloc(&s->w2b, kHidden * kHidden * 2) != hipSuccess ||
      hipMalloc(&s->w2bt, kHidden * kHidden * 2) != hipSuccess ||
      hipMalloc(&s->adam_m, kNParams * 4) != hipSuccess || hipMalloc(&s->adam_v, kNParams * 4) != hipSuccess ||
      hipMalloc(&s->wtab, 64 * 16) != hipSuccess ||
      hipMalloc(&s->partials, s->max_blocks * kNParams * 4) != hipSuccess ||
      hipMalloc(&s->loss_part, s->max_blocks * 4) != hipSuccess ||
      hipMalloc(&s->scratch, (kNParams + 1) * 8) != hipSuccess ||
      hipMalloc(&s->stage, size_t(kMaxSlices) * (kNParams + 1) * 8) != hipSuccess) {
    free_surrogate(s);
    return fail(AICDF_ENOMEM, "device allocation for the surrogate failed");
  }
  // the w feature: the library's 16-row cubic dyadic table in FP32
  std::vector<double> tab = build_dyadic_table(16, 3);
  std::vector<float> rows(64 * 4, 0.0f);
  for (int e = 0; e < 16; ++e)
    for (int j = 0; j < 4; ++j) rows[e * 4 + j] = float(tab[e * 4 + j]);
  if (hipMemcpy(s->wtab, rows.data(), rows.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(s->adam_m, 0, kNParams * 4) != hipSuccess || hipMemset(s->adam_v, 0, kNParams * 4) != hipSuccess) {
    free_surrogate(s);
    return fail(AICDF_EHIP, "initialising the surrogate failed");
  }
  *out = s;
  return AICDF_OK;
}

aicdf_status upload_params(aicdf_surrogate* s, const float* host) {
  AICDF_HIP(hipMemcpy(s->params, host, kNParams * 4, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(w2_refresh_kernel, dim3(16), dim3(256), 0, 0, s->params, s->w2b, s->w2bt);
  AICDF_HIP(hipGetLastError());
  AICDF_HIP(hipMemset(s->adam_m, 0, kNParams * 4));
  AICDF_HIP(hipMemset(s->adam_v, 0, kNParams * 4));
  AICDF_HIP(hipDeviceSynchronize());
  s->step = 0;
  return AICDF_OK;
}

}  // namespace

// Internal accessors for the CIR level kernel.
namespace aicdf {
const float* surrogate_params(const aicdf_surrogate* s) { return s->params; }
const uint16_t* surrogate_w2b(const aicdf_surrogate* s) { return s->w2b; }
const float* surrogate_wtab(const aicdf_surrogate* s) { return s->wtab; }
void surrogate_range(const aicdf_surrogate* s, double* nu, double* lo, double* hi, int* dev) {
  *nu = s->nu;
  *lo = s->lo;
  *hi = s->hi;
  *dev = s->device;
}
}  // namespace aicdf

extern "C" aicdf_status aicdf_surrogate_create(double nu, double lo, double hi, uint64_t seed, aicdf_surrogate** out) {
  if (!out) return fail(AICDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!(nu > 0.0) || !(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi))
    return fail(AICDF_EINVAL, "need nu > 0 and loglam_lo < loglam_hi");
  aicdf_surrogate* s = nullptr;
  aicdf_status st = alloc_surrogate(nu, lo, hi, &s);
  if (st != AICDF_OK) return st;
  std::vector<float> p(kNParams);
  uint64_t state = seed;
  auto unif = [&](double a) { return float(a * (2.0 * double(splitmix64(state) >> 11) * 0x1p-53 - 1.0)); };
  for (int i = 0; i < 128; ++i) p[kOffW1 + i] = unif(1.0 / std::sqrt(2.0));
  for (int i = 0; i < 64; ++i) p[kOffB1 + i] = unif(1.0 / std::sqrt(2.0));
  for (int i = 0; i < 4096; ++i) p[kOffW2 + i] = unif(1.0 / 8.0);
  for (int i = 0; i < 64; ++i) p[kOffB2 + i] = unif(1.0 / 8.0);
  for (int i = 0; i < 64; ++i) p[kOffW3 + i] = unif(1.0 / 8.0);
  p[kOffB3] = 0.0f;
  if ((st = upload_params(s, p.data())) != AICDF_OK) {
    free_surrogate(s);
    return st;
  }
  *out = s;
  return ok();
}

extern "C" void aicdf_surrogate_destroy(aicdf_surrogate* s) { free_surrogate(s); }

extern "C" aicdf_status aicdf_surrogate_set_params(aicdf_surrogate* s, const float* host, size_t n) {
  if (!s || !host) return fail(AICDF_EINVAL, "NULL argument");
  if (n != size_t(kNParams)) return fail(AICDF_EINVAL, "need %d parameters, got %zu", kNParams, n);
  aicdf_status st = check_dev(s);
  if (st != AICDF_OK) return st;
  if ((st = upload_params(s, host)) != AICDF_OK) return st;
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_get_params(const aicdf_surrogate* s, float* host, size_t n) {
  if (!s || !host) return fail(AICDF_EINVAL, "NULL argument");
  if (n < size_t(kNParams)) return fail(AICDF_EINVAL, "need room for %d parameters", kNParams);
  aicdf_status st = check_dev(s);
  if (st != AICDF_OK) return st;
  AICDF_HIP(hipDeviceSynchronize());
  AICDF_HIP(hipMemcpy(host, s->params, kNParams * 4, hipMemcpyDeviceToHost));
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_info(const aicdf_surrogate* s, double* nu, double* lo, double* hi) {
  if (!s) return fail(AICDF_EINVAL, "surrogate is NULL");
  if (nu) *nu = s->nu;
  if (lo) *lo = s->lo;
  if (hi) *hi = s->hi;
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_forward(const aicdf_surrogate* s, size_t n, const float* u,
                                                const float* loglam, float* p, void* stream) {
  if (!s) return fail(AICDF_EINVAL, "surrogate is NULL");
  if (n == 0) return ok();
  if (!u || !loglam || !p) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * 4, p, n * 4) || overlaps(loglam, n * 4, p, n * 4)) return fail(AICDF_EALIAS, "p overlaps an input");
  aicdf_status st = check_dev(s);
  if (st != AICDF_OK) return st;
  const size_t need = (n + 255) / 256;
  const unsigned grid = unsigned(need < 4096 ? need : 4096);
  const float inv_span2 = float(2.0 / (s->hi - s->lo));
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), s->params,
                     s->w2b, reinterpret_cast<const f32x4*>(s->wtab), n, u, loglam, p, float(s->lo), inv_span2);
  AICDF_HIP(hipGetLastError());
  return ok();
}

namespace {
// One gradient evaluation over samples [first, first+count) of the permuted
// data; mode 0 leaves the summed gradient in scratch, mode 1 applies Adam.
aicdf_status grad_pass(aicdf_surrogate* s, const float* u, const float* ll, const float* t, size_t n_data,
                       uint64_t pa, uint64_t pb, size_t first, size_t count, float inv_batch, int adam, float lr,
                       hipStream_t st) {
  const unsigned nb = unsigned((count + kTrainWave - 1) / kTrainWave);
  if (nb > s->max_blocks) return fail(AICDF_ERANGE, "batch too large");
  const float inv_span2 = float(2.0 / (s->hi - s->lo));
  hipLaunchKernelGGL(mlp_train_kernel, dim3(nb), dim3(kTrainWave), 0, st, s->params, s->w2b, s->w2bt,
                     reinterpret_cast<const f32x4*>(s->wtab), u, ll, t, n_data, pa, pb, first, count, inv_batch,
                     float(s->lo), inv_span2, s->partials, s->loss_part);
  float bc1 = 1.0f, bc2 = 1.0f;
  if (adam) {
    ++s->step;
    bc1 = float(1.0 - std::pow(0.9, double(s->step)));
    bc2 = float(1.0 - std::pow(0.999, double(s->step)));
  }
  const unsigned slices = std::min(kMaxSlices, (nb + kSliceRows - 1) / kSliceRows);
  const unsigned rows = (nb + slices - 1) / slices;
  hipLaunchKernelGGL(mlp_slice_sum_kernel, dim3((kNParams + 1 + 255) / 256, slices), dim3(256), 0, st, s->partials,
                     s->loss_part, nb, rows, s->stage);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNParams + 1 + 255) / 256), dim3(256), 0, st, s->stage, slices,
                     s->scratch, s->params, s->adam_m, s->adam_v, s->w2b, s->w2bt, adam, lr, bc1, bc2);
  AICDF_HIP(hipGetLastError());
  return AICDF_OK;
}
}  // namespace

extern "C" aicdf_status aicdf_surrogate_loss_grad(const aicdf_surrogate* sc, size_t n, const float* u,
                                                  const float* loglam, const float* target, double* host_loss,
                                                  float* host_grads, void* stream) {
  auto* s = const_cast<aicdf_surrogate*>(sc);
  if (!s || !u || !loglam || !target) return fail(AICDF_EINVAL, "NULL argument");
  if (n == 0 || n > kMaxTrainBlocks * kTrainWave)
    return fail(AICDF_ERANGE, "n must be in [1, %zu]", kMaxTrainBlocks * kTrainWave);
  aicdf_status st = check_dev(s);
  if (st != AICDF_OK) return st;
  auto hs = static_cast<hipStream_t>(stream);
  AICDF_HIP(hipMemsetAsync(s->scratch, 0, (kNParams + 1) * 8, hs));
  if ((st = grad_pass(s, u, loglam, target, n, 1, 0, 0, n, float(1.0 / double(n)), 0, 0.0f, hs)) != AICDF_OK)
    return st;
  std::vector<double> g(kNParams + 1);
  AICDF_HIP(hipMemcpyAsync(g.data(), s->scratch, (kNParams + 1) * 8, hipMemcpyDeviceToHost, hs));
  AICDF_HIP(hipStreamSynchronize(hs));
  if (host_grads)
    for (int i = 0; i < kNParams; ++i) host_grads[i] = float(g[i]);
  if (host_loss) *host_loss = g[kNParams] / double(n);
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_make_data(const aicdf_surrogate* s, uint64_t seed, size_t n, float* u,
                                                  float* loglam, float* target, void* stream) {
  if (!s) return fail(AICDF_EINVAL, "surrogate is NULL");
  if (n == 0) return ok();
  if (!u || !loglam || !target) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * 4, loglam, n * 4) || overlaps(u, n * 4, target, n * 4) || overlaps(loglam, n * 4, target, n * 4))
    return fail(AICDF_EALIAS, "output buffers overlap");
  aicdf_status st = check_dev(s);
  if (st != AICDF_OK) return st;
  const size_t need = (n + 255) / 256;
  const unsigned grid = unsigned(need < 16384 ? need : 16384);
  hipLaunchKernelGGL(make_data_kernel, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream), uint32_t(seed),
                     uint32_t(seed >> 32), n, s->nu, float(s->lo), float(s->hi), u, loglam, target);
  AICDF_HIP(hipGetLastError());
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_train(aicdf_surrogate* s, size_t n, const float* u, const float* loglam,
                                              const float* target, uint32_t epochs, uint32_t batch, float lr,
                                              uint64_t seed, double* host_loss, void* stream) {
  if (!s || !u || !loglam || !target) return fail(AICDF_EINVAL, "NULL argument");
  if (n == 0 || epochs == 0) return fail(AICDF_EINVAL, "need n > 0 and epochs > 0");
  if (batch == 0 || batch % 256 || batch > kMaxTrainBlocks * kTrainWave)
    return fail(AICDF_EINVAL, "batch must be a multiple of 256 <= %zu", kMaxTrainBlocks * kTrainWave);
  if (!(lr > 0.0f)) return fail(AICDF_EINVAL, "lr must be > 0");
  aicdf_status st = check_dev(s);
  if (st != AICDF_OK) return st;
  auto hs = static_cast<hipStream_t>(stream);
  const size_t steps_per_epoch = (n + batch - 1) / batch;
  const double total = double(steps_per_epoch) * epochs;
  uint64_t state = seed ^ 0xC0FFEE;
  double step_i = 0.0;
  double last_loss = 0.0;
  for (uint32_t ep = 0; ep < epochs; ++ep) {
    // pseudo-random permutation i -> (a i + b) mod n with gcd(a, n) = 1
    uint64_t a = 1, b = 0;
    if (n > 1) {
      do {
        a = splitmix64(state) % n;
      } while (a == 0 || gcd64(a, n) != 1);
      b = splitmix64(state) % n;
    }
    AICDF_HIP(hipMemsetAsync(s->scratch + kNParams, 0, 8, hs));
    for (size_t k = 0; k < steps_per_epoch; ++k, step_i += 1.0) {
      const size_t first = k * batch;
      const size_t count = std::min<size_t>(batch, n - first);
      const float lr_k = float(lr * (0.05 + 0.95 * 0.5 * (1.0 + std::cos(M_PI * step_i / total))));
      if ((st = grad_pass(s, u, loglam, target, n, a, b, first, count, float(1.0 / double(count)), 1, lr_k, hs)) !=
          AICDF_OK)
        return st;
    }
    double lsum = 0.0;
    AICDF_HIP(hipMemcpyAsync(&lsum, s->scratch + kNParams, 8, hipMemcpyDeviceToHost, hs));
    AICDF_HIP(hipStreamSynchronize(hs));
    last_loss = lsum / double(n);
  }
  if (host_loss) *host_loss = last_loss;
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_save(const aicdf_surrogate* s, const char* path) {
  if (!s || !path) return fail(AICDF_EINVAL, "NULL argument");
  std::vector<float> p(kNParams);
  aicdf_status st = aicdf_surrogate_get_params(s, p.data(), p.size());
  if (st != AICDF_OK) return st;
  std::ofstream f(path, std::ios::binary);
  if (!f) return fail(AICDF_EIO, "cannot open %s", path);
  const char magic[8] = {'A', 'I', 'C', 'D', 'F', 'S', 'U', 'R'};
  const uint32_t version = kFileVersion, np = kNParams;
  f.write(magic, 8);
  f.write(reinterpret_cast<const char*>(&version), 4);
  f.write(reinterpret_cast<const char*>(&np), 4);
  f.write(reinterpret_cast<const char*>(&s->nu), 8);
  f.write(reinterpret_cast<const char*>(&s->lo), 8);
  f.write(reinterpret_cast<const char*>(&s->hi), 8);
  f.write(reinterpret_cast<const char*>(p.data()), kNParams * 4);
  if (!f) return fail(AICDF_EIO, "write to %s failed", path);
  return ok();
}

extern "C" aicdf_status aicdf_surrogate_load(const char* path, aicdf_surrogate** out) {
  if (!path || !out) return fail(AICDF_EINVAL, "NULL argument");
  *out = nullptr;
  std::ifstream f(path, std::ios::binary);
  if (!f) return fail(AICDF_EIO, "cannot open %s", path);
  char magic[8];
  uint32_t version = 0, np = 0;
  double nu = 0, lo = 0, hi = 0;
  f.read(magic, 8);
  f.read(reinterpret_cast<char*>(&version), 4);
  f.read(reinterpret_cast<char*>(&np), 4);
  f.read(reinterpret_cast<char*>(&nu), 8);
  f.read(reinterpret_cast<char*>(&lo), 8);
  f.read(reinterpret_cast<char*>(&hi), 8);
  if (!f || std::memcmp(magic, "AICDFSUR", 8) != 0 || version != kFileVersion || np != uint32_t(kNParams))
    return fail(AICDF_EIO, "%s is not a surrogate file of this version", path);
  std::vector<float> p(kNParams);
  f.read(reinterpret_cast<char*>(p.data()), kNParams * 4);
  if (!f) return fail(AICDF_EIO, "%s is truncated", path);
  aicdf_surrogate* s = nullptr;
  aicdf_status st = alloc_surrogate(nu, lo, hi, &s);
  if (st != AICDF_OK) return st;
  if ((st = upload_params(s, p.data())) != AICDF_OK) {
    free_surrogate(s);
    return st;
  }
  *out = s;
  return ok();
}
