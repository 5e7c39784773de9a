// Wave-level forward pass of the surrogate network on the CDNA4 matrix cores.
//
// One 64-lane wave evaluates 64 samples (lane s owns sample s):
//   h1 = silu(W1 [w, g] + b1)            64 x 2, VALU (FP32)
//   a2 = W2 bf16(h1) + b2                64 x 64, BF16 MFMA, FP32 sums
//   P~ = w + W3 . silu(a2) + b3          64, VALU + one cross-half shuffle
// Layer 2 is computed transposed, A2^T = W2 . H1^T, with
// v_mfma_f32_32x32x16_bf16 (M = output unit, N = sample, K = input unit):
//   A operand, lane l: W2[32 mt + l%32][16 kt + 8 (l/32) + 0..7]   (registers)
//   B operand, lane l: bf16(h1)[sample 32 nt + l%32][16 kt + 8 (l/32) + 0..7]
//   result,    lane l: a2[sample 32 nt + l%32][32 mt + 8 (j/4) + 4 (l/32) + j%4]
// for tiles mt, nt in {0,1}, kt in {0..3}, j in {0..15} (layouts checked on
// the device against an exact integer product).  Every lane therefore needs
// the inputs of samples l%32 and l%32 + 32 (one xor-32 shuffle) and computes
// the 64 layer-1 values its B fragments hold; after layer 2 it holds 32
// output units of each of those two samples, and the lane pair (l, l^32)
// completes the layer-3 dot product with one more shuffle.
#pragma once

#include "device_common.hpp"

namespace aicdf {

constexpr int kHidden = 64;
constexpr int kNParams = kHidden * 2 + kHidden + kHidden * kHidden + kHidden + kHidden + 1;  // 4417
// offsets in the flat parameter vector
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 4288, kOffW3 = 4352, kOffB3 = 4416;

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using f32x16 = float __attribute__((ext_vector_type(16)));
using f32x2 = vec_t<float, 2>;

// Per work-group copy of the small parameters (LDS).
struct MlpLds {
  f32x4 u1[kHidden];  // W1[k][0], W1[k][1], b1[k], 0
  f32x2 u2[kHidden];  // b2[m], W3[m]
  float b3;
};

__device__ __forceinline__ void mlp_stage_params(MlpLds& L, const float* __restrict__ p, int tid, int nthreads) {
  for (int k = tid; k < kHidden; k += nthreads) {
    L.u1[k] = f32x4{p[kOffW1 + 2 * k], p[kOffW1 + 2 * k + 1], p[kOffB1 + k], 0.0f};
    L.u2[k] = f32x2{p[kOffB2 + k], p[kOffW3 + k]};
  }
  if (tid == 0) L.b3 = p[kOffB3];
}

// silu(t) = t / (1 + e^-t) with the hardware exponential and reciprocal.
__device__ __forceinline__ float mlp_sigmoid(float t) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-t));
}
__device__ __forceinline__ float mlp_silu(float t) { return t * mlp_sigmoid(t); }

__device__ __forceinline__ __bf16 to_bf16(float x) { return __builtin_bit_cast(__bf16, f32_to_bf16_bits(x)); }

// The W2 A-operand fragments of this lane from the BF16 row-major [out][in]
// copy in global memory (16-byte loads; kept in registers).
__device__ __forceinline__ void mlp_load_w2(const uint16_t* __restrict__ w2b, bf16x8 (&A)[2][4]) {
  const int l = __lane_id(), r = l & 31, half = l >> 5;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      A[mt][kt] = *reinterpret_cast<const bf16x8*>(w2b + (32 * mt + r) * kHidden + 16 * kt + 8 * half);
}

// Layer-1 B fragments for samples (l%32, l%32+32).  ws/gs: inputs of those.
__device__ __forceinline__ void mlp_layer1(const MlpLds& L, const float (&ws)[2], const float (&gs)[2],
                                           bf16x8 (&B)[2][4]) {
  const int half = __lane_id() >> 5;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const f32x4 c = L.u1[16 * kt + 8 * half + i];
        B[nt][kt][i] = to_bf16(mlp_silu(fmaf(c[0], ws[nt], fmaf(c[1], gs[nt], c[2]))));
      }
}

// Layer 2 on MFMA: acc[mt][nt] = A2^T tile (without b2).
__device__ __forceinline__ void mlp_layer2(const bf16x8 (&A)[2][4], const bf16x8 (&B)[2][4], f32x16 (&acc)[2][2]) {
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 c = {};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mt][kt], B[nt][kt], c, 0, 0, 0);
      acc[mt][nt] = c;
    }
}

// Output unit held in slot (mt, j) by a lane of half `half`.
__device__ __forceinline__ int mlp_unit(int mt, int j, int half) { return 32 * mt + 8 * (j >> 2) + 4 * half + (j & 3); }

// Full forward pass; every lane of the wave must call it.  Returns P~ of the
// lane's own sample.
__device__ __forceinline__ float mlp_wave_forward(const MlpLds& L, const bf16x8 (&A)[2][4], float w, float g) {
  // the parameters are read from LDS at every call: hoisted out of a caller's
  // loop they would hold ~200 VGPRs and leave one wave per SIMD
  asm volatile("" ::: "memory");
  const int l = __lane_id(), half = l >> 5;
  const float wo = __shfl_xor(w, 32), go = __shfl_xor(g, 32);
  const float ws[2] = {half ? wo : w, half ? w : wo};
  const float gs[2] = {half ? go : g, half ? g : go};
  bf16x8 B[2][4];
  mlp_layer1(L, ws, gs, B);
  // layer 2 and 3 one (sample tile, unit tile) at a time: the sums of one
  // sample tile run over mt, then j, as in a single pass
  float part[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    float p = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x16 acc = {};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mt][kt], B[nt][kt], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const f32x2 q = L.u2[mlp_unit(mt, j, half)];
        p = fmaf(q[1], mlp_silu(acc[j] + q[0]), p);
      }
    }
    part[nt] = p + __shfl_xor(p, 32);
  }
  return w + (half ? part[1] : part[0]) + L.b3;
}

// W2 in LDS for mlp_wave_forward_one: BF16 rows of kHidden inputs padded to
// kW2Stride, so that the 16-byte fragment reads of 8 consecutive rows fall in
// distinct banks.
constexpr int kW2Stride = kHidden + 8;

__device__ __forceinline__ void mlp_stage_w2(uint16_t* __restrict__ w2s, const uint16_t* __restrict__ w2b, int tid,
                                             int nthreads) {
  for (int c = tid; c < kHidden * kHidden / 8; c += nthreads) {
    const int row = c / (kHidden / 8), col = 8 * (c % (kHidden / 8));
    *reinterpret_cast<bf16x8*>(w2s + row * kW2Stride + col) =
        *reinterpret_cast<const bf16x8*>(w2b + row * kHidden + col);
  }
}

// Per-wave LDS exchange of mlp_wave_forward_one.
struct alignas(16) MlpXchg {
  uint16_t h[kHidden];  // bf16 bits of the layer-1 values
  float s[kHidden];     // silu of the layer-2 values
};

// Forward pass of ONE sample held by the whole wave (w and g equal in every
// lane, as when all lanes follow one path): the arithmetic of
// mlp_wave_forward for that sample, bit for bit, with the per-unit work
// spread over the lanes instead of repeated in each.  Layer 1: lane l
// computes unit l; the BF16 values meet in LDS, from which every lane reads
// its B fragments (all 32 sample columns are then the same, so only the
// nt = 0 tiles are computed).  After layer 2 the 32 lanes of a half hold the
// same 32 output units; lane l takes the slot (mt, j) = (l%32 / 16, l%16) of
// its half, so every unit's silu is evaluated once, and the values meet in
// LDS again.  Each lane then runs both halves' FMA chains in the order of
// mlp_wave_forward.  Every lane of the wave must call it, with wave-uniform
// control flow.
__device__ __forceinline__ float mlp_wave_forward_one(const MlpLds& L, MlpXchg& X, const uint16_t* __restrict__ w2s,
                                                      float w, float g) {
  asm volatile("" ::: "memory");  // parameters from LDS at every call (as above)
  const int l = __lane_id(), half = l >> 5, r = l & 31;
  // the W2 fragments of mlp_load_w2, from the padded LDS copy (the caller
  // keeps no registers for them between calls)
  bf16x8 A[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      A[mt][kt] = *reinterpret_cast<const bf16x8*>(w2s + (32 * mt + r) * kW2Stride + 16 * kt + 8 * half);
  const f32x4 c = L.u1[l];
  X.h[l] = f32_to_bf16_bits(mlp_silu(fmaf(c[0], w, fmaf(c[1], g, c[2]))));
  __syncwarp();
  bf16x8 B[4];
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) B[kt] = *reinterpret_cast<const bf16x8*>(&X.h[16 * kt + 8 * half]);
  f32x16 acc[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 a = {};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mt][kt], B[kt], a, 0, 0, 0);
    acc[mt] = a;
  }
  // acc[r / 16][r % 16] by a select tree on the bits of r
  float t[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) t[j] = (r & 16) ? acc[1][j] : acc[0][j];
#pragma unroll
  for (int j = 0; j < 8; ++j) t[j] = (r & 8) ? t[j + 8] : t[j];
#pragma unroll
  for (int j = 0; j < 4; ++j) t[j] = (r & 4) ? t[j + 4] : t[j];
#pragma unroll
  for (int j = 0; j < 2; ++j) t[j] = (r & 2) ? t[j + 2] : t[j];
  const float v = (r & 1) ? t[1] : t[0];
  const int u = mlp_unit(r >> 4, r & 15, half);
  X.s[u] = mlp_silu(v + L.u2[u][0]);
  __syncwarp();
  float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int u0 = mlp_unit(mt, j, 0), u1 = mlp_unit(mt, j, 1);
      p0 = fmaf(L.u2[u0][1], X.s[u0], p0);
      p1 = fmaf(L.u2[u1][1], X.s[u1], p1);
    }
  __syncwarp();  // X is rewritten by the next call
  return w + (p0 + p1) + L.b3;
}

// The input feature g of the network.
__device__ __forceinline__ float mlp_g(float loglam, float lo, float inv_span2) {
  return fmaf(loglam - lo, inv_span2, -1.0f);
}

}  // namespace aicdf
