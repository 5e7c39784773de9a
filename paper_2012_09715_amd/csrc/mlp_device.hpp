// Wave-level forward pass of the surrogate network on the CDNA4 matrix cores.
//
// One 64-lane wave evaluates 64 samples (lane s owns sample s):
//   a1 = W1 [w, g] + b1                  64 x 2, split-BF16 MFMA (below)
//   h1 = relu(a1)                        VALU, rounded to BF16
//   a2 = W2 bf16(h1) + b2                64 x 64, BF16 MFMA, FP32 sums
//   P~ = w + W3 . relu(a2) + b3          64, VALU + one cross-half shuffle
// Layer 2 is computed transposed, A2^T = W2 . H1^T, with
// v_mfma_f32_32x32x16_bf16 (M = output unit, N = sample, K = input unit):
//   A operand, lane l: W2[32 mt + l%32][16 kt + 8 (l/32) + 0..7]   (registers)
//   B operand, lane l: bf16(h1)[sample 32 nt + l%32][16 kt + 8 (l/32) + 0..7]
//   result,    lane l: a2[sample 32 nt + l%32][32 mt + 8 (j/4) + 4 (l/32) + j%4]
// for tiles mt, nt in {0,1}, kt in {0..3}, j in {0..15} (layouts checked on
// the device against an exact integer product); the accumulators start at
// b2.  Layer 1 is one more product of the same shape with K = 16: row r of
// its A operand holds, in K slots 0..7, the weights of hidden unit u1(r) as
// BF16 parts (Ww_hi, Ww_lo, Ww_hi, Wg_hi, Wg_lo, Wg_hi, b_hi, b_lo), and
// the B column of a sample holds (w_hi, w_hi, w_lo, g_hi, g_hi, g_lo, 1, 1)
// (x_hi = bf16(x), x_lo = bf16(x - x_hi); the A rows are zero in slots
// 8..15, where the B columns then may hold any finite values), so that
// a1 = W1 [w, g] + b1 to about 2^-16 relative with exact products.  The
// order u1 of the rows puts each lane's layer-1 results exactly where its
// layer-2 B fragments need them: lane l's result slot j of tile (mt, nt) is
// hidden unit 16 kt + 8 (l/32) + i with kt = 2 mt + j/8, i = j%8.  Every
// lane needs the inputs of samples l%32 and l%32 + 32 (one xor-32 shuffle);
// after layer 2 it holds 32 output units of each of those two samples, and
// the lane pair (l, l^32) completes the layer-3 dot product with one more
// shuffle.
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

// Output unit held in slot (mt, j) by a lane of half `half` (layer 2).
__device__ __forceinline__ int mlp_unit(int mt, int j, int half) { return 32 * mt + 8 * (j >> 2) + 4 * half + (j & 3); }

// Hidden unit of row r = 32 mt + 8 q + 4 h + jj of the layer-1 A operand:
// 16 (2 mt + q/2) + 8 h + 4 (q%2) + jj (see the file header).
__device__ __forceinline__ int mlp_unit1(int r) {
  const int mt = r >> 5, q = (r >> 3) & 3, h = (r >> 2) & 1, jj = r & 3;
  return 16 * (2 * mt + (q >> 1)) + 8 * h + 4 * (q & 1) + jj;
}

// Per work-group copy of the small parameters (LDS).
struct MlpLds {
  bf16x8 a1[2][64];     // layer-1 A fragments in split BF16 by tile and lane
                        // (zero for lanes 32..63, K slots 8..15)
  float b2s[2][2][16];  // b2 of unit mlp_unit(mt, j, half), as [mt][half][j]
  float w3s[2][2][16];  // W3 likewise
  float b3;
};

__device__ __forceinline__ __bf16 to_bf16(float x) { return __builtin_bit_cast(__bf16, f32_to_bf16_bits(x)); }

// x = hi + lo + r: hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32).
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = to_bf16(x);
  lo = to_bf16(x - __uint_as_float(uint32_t(__builtin_bit_cast(uint16_t, hi)) << 16));
}

__device__ __forceinline__ void mlp_stage_params(MlpLds& L, const float* __restrict__ p, int tid, int nthreads) {
  for (int k = tid; k < kHidden; k += nthreads) {
    const int u = mlp_unit1(k);
    __bf16 wh, wl, gh, gl, bh, bl;
    split_bf16(p[kOffW1 + 2 * u], wh, wl);
    split_bf16(p[kOffW1 + 2 * u + 1], gh, gl);
    split_bf16(p[kOffB1 + u], bh, bl);
    const __bf16 zero = to_bf16(0.0f);
    L.a1[k >> 5][k & 31] = bf16x8{wh, wl, wh, gh, gl, gh, bh, bl};
    L.a1[k >> 5][32 + (k & 31)] = bf16x8{zero, zero, zero, zero, zero, zero, zero, zero};
    const int mt = k >> 5, half = (k >> 4) & 1, j = k & 15;
    L.b2s[mt][half][j] = p[kOffB2 + mlp_unit(mt, j, half)];
    L.w3s[mt][half][j] = p[kOffW3 + mlp_unit(mt, j, half)];
  }
  if (tid == 0) L.b3 = p[kOffB3];
}

// The activation of both hidden layers, relu(t) = max(t, 0): one VALU
// operation and no transcendental function (with t / (1 + e^-t) the
// exponential and the reciprocal of the 128 activations per sample bounded
// the surrogate levels), and its derivative, taken as 0 at t = 0.  The
// maximum is taken on the bit patterns as signed integers, which orders
// finite floats of either sign against +0 as the float maximum does (every
// negative float, -0 included, is a negative integer); a float maximum
// would first quiet possible signalling NaNs of matrix-core results, one
// more instruction per activation.
__device__ __forceinline__ float mlp_act(float t) { return __int_as_float(max(__float_as_int(t), 0)); }
__device__ __forceinline__ float mlp_act_grad(float t) { return t > 0.0f ? 1.0f : 0.0f; }

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

// A 64 x 64 x 64 product on MFMA (the training kernel's backward products):
// acc[mt][nt] = the (mt, nt) tile of A B, accumulators from zero.
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

// The layer-1 B fragment of one sample: (w_hi, w_hi, w_lo, g_hi, g_hi,
// g_lo, 1, 1).  In lanes 32..63 (K slots 8..15) it meets the zero A slots,
// so those lanes may pass any finite w and g.
__device__ __forceinline__ bf16x8 mlp_input_frag(float w, float g) {
  __bf16 wh, wl, gh, gl;
  split_bf16(w, wh, wl);
  split_bf16(g, gh, gl);
  const __bf16 one = to_bf16(1.0f);
  return bf16x8{wh, wh, wl, gh, gh, gl, one, one};
}

// Layer-1 A fragment of tile mt (zero in lanes 32..63).
__device__ __forceinline__ bf16x8 mlp_w1_frag(const MlpLds& L, int mt) { return L.a1[mt][__lane_id()]; }

// bf16(relu(a)), bf16(relu(b)) packed in one word: one two-value conversion
// and one packed 16-bit integer maximum (the rounding commutes with relu: a
// negative value rounds to a BF16 of the same sign, which the integer
// maximum with 0 then clears, -0 included).
__device__ __forceinline__ uint32_t mlp_act_bf16_pair(float a, float b) {
  using f32x2v = float __attribute__((ext_vector_type(2)));
  using s16x2 = short __attribute__((ext_vector_type(2)));
  using bf16x2 = __bf16 __attribute__((ext_vector_type(2)));
  const bf16x2 v = __builtin_convertvector(f32x2v{a, b}, bf16x2);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), s16x2{0, 0}));
}

// Layer-2 B fragments kt = 2 mt, 2 mt + 1 from the layer-1 accumulator of
// tile mt: B[kt][i] = bf16(relu(a1 slot 8 (kt%2) + i)).
__device__ __forceinline__ void mlp_h1_frags(const f32x16& a1, int mt, bf16x8 (&B)[4]) {
  using u32x4 = uint32_t __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    u32x4 q;
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = mlp_act_bf16_pair(a1[8 * k + 2 * i], a1[8 * k + 2 * i + 1]);
    B[2 * mt + k] = __builtin_bit_cast(bf16x8, q);
  }
}

// Layer 1 of one sample tile: the B fragments of layer 2 (one layer-1
// accumulator tile live at a time).
__device__ __forceinline__ void mlp_layer1_mfma(const bf16x8& W0, const bf16x8& W1f, const bf16x8& X,
                                                bf16x8 (&B)[4]) {
  mlp_h1_frags(__builtin_amdgcn_mfma_f32_32x32x16_bf16(W0, X, f32x16{}, 0, 0, 0), 0, B);
  mlp_h1_frags(__builtin_amdgcn_mfma_f32_32x32x16_bf16(W1f, X, f32x16{}, 0, 0, 0), 1, B);
}

// The layer-2 accumulator start of tile mt: b2 of the lane's 16 units.
__device__ __forceinline__ f32x16 mlp_b2_acc(const MlpLds& L, int mt, int half) {
  const f32x4* b = reinterpret_cast<const f32x4*>(L.b2s[mt][half]);
  const f32x4 b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];
  return f32x16{b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3],
                b2[0], b2[1], b2[2], b2[3], b3[0], b3[1], b3[2], b3[3]};
}

// Full forward pass; every lane of the wave must call it.  Returns P~ of the
// lane's own sample.
__device__ __forceinline__ float mlp_wave_forward(const MlpLds& L, const bf16x8 (&A)[2][4], float w, float g) {
  // the parameters are read from LDS at every call: hoisted out of a caller's
  // loop they would hold many VGPRs and leave fewer waves per SIMD
  asm volatile("" ::: "memory");
  const int l = __lane_id(), half = l >> 5;
  const float wo = __shfl_xor(w, 32), go = __shfl_xor(g, 32);
  const bf16x8 X0 = mlp_input_frag(w, g);    // samples 0..31 (lanes 0..31)
  const bf16x8 X1 = mlp_input_frag(wo, go);  // samples 32..63
  const bf16x8 W0 = mlp_w1_frag(L, 0), W1f = mlp_w1_frag(L, 1);
  // layers 2 and 3 one sample tile at a time: the sums of one sample tile
  // run over mt, then j, as in a single pass
  float part[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    bf16x8 B[4];
    mlp_layer1_mfma(W0, W1f, nt ? X1 : X0, B);
    float p = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x16 acc = mlp_b2_acc(L, mt, half);
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mt][kt], B[kt], acc, 0, 0, 0);
      const f32x4* w3 = reinterpret_cast<const f32x4*>(L.w3s[mt][half]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 c = w3[q];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) p = fmaf(c[jj], mlp_act(acc[4 * q + jj]), p);
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
  float s[kHidden];  // activations of the layer-2 values
};

// Forward pass of ONE sample held by the whole wave (w and g equal in every
// lane, as when all lanes follow one path): the arithmetic of
// mlp_wave_forward for that sample, bit for bit, with the layer-3 work
// spread over the lanes instead of repeated in each.  The sample fills every
// column of the layer-1 and layer-2 products (the same matrix-core
// instructions on the same operands give the same values; only the nt = 0
// tiles are computed).  After layer 2 the 32 lanes of a half hold the same
// 32 output units; lane l takes the slot (mt, j) = (l%32 / 16, l%16) of its
// half, so every unit's activation is evaluated once, and the values meet in
// LDS.  Each lane then runs both halves' FMA chains in the order of
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
  bf16x8 B[4];
  mlp_layer1_mfma(mlp_w1_frag(L, 0), mlp_w1_frag(L, 1), mlp_input_frag(w, g), B);
  f32x16 acc[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f32x16 a = mlp_b2_acc(L, mt, half);
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
  X.s[mlp_unit(r >> 4, r & 15, half)] = mlp_act(v);
  __syncwarp();
  float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      p0 = fmaf(L.w3s[mt][0][j], X.s[mlp_unit(mt, j, 0)], p0);
      p1 = fmaf(L.w3s[mt][1][j], X.s[mlp_unit(mt, j, 1)], p1);
    }
  __syncwarp();  // X is rewritten by the next call
  return w + (p0 + p1) + L.b3;
}

// The input feature g of the network.
__device__ __forceinline__ float mlp_g(float loglam, float lo, float inv_span2) {
  return fmaf(loglam - lo, inv_span2, -1.0f);
}

}  // namespace aicdf
