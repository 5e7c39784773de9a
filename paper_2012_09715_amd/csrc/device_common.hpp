// Device-side building blocks shared by the kernels of libaicdf (gfx950):
// Philox-4x32-10, the uniform grids, output rounding, and the exact FP64
// inverse normal CDF.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aicdf {

template <typename T, int N>
using vec_t = T __attribute__((ext_vector_type(N)));

using f32x4 = vec_t<float, 4>;
using f64x2 = vec_t<double, 2>;
using u32x4 = vec_t<uint32_t, 4>;
using u16x4 = vec_t<uint16_t, 4>;

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the round keys bumped by the Weyl constants.
__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = c0 * 0xD2511F53u, hi0 = __umulhi(c0, 0xD2511F53u);
    const uint32_t lo1 = c2 * 0xCD9E8D57u, hi1 = __umulhi(c2, 0xCD9E8D57u);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return u32x4{c0, c1, c2, c3};
}

// u24 grid: odd multiples of 2^-24 from the top 23 bits of a word (exact).
__device__ __forceinline__ float u24_from_word(uint32_t w) {
  return (float(w >> 9) + 0.5f) * 0x1p-23f;
}

// u53 grid: ((double)k + 0.5) 2^-53, k = top 53 bits of hi:lo, RNE; the
// single value rounding to 1 becomes 1 - 2^-53.
__device__ __forceinline__ double u53_from_words(uint32_t hi, uint32_t lo) {
  const uint64_t w = (uint64_t(hi) << 32) | lo;
  const double k = double(w >> 11);
  double u = __dmul_rn(__dadd_rn(k, 0.5), 0x1p-53);
  return u == 1.0 ? 1.0 - 0x1p-53 : u;
}

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN): the gfx950
// conversion instruction (v_cvt_pk_bf16_f32, two values per instruction when
// the compiler pairs them) instead of integer rounding with a NaN branch.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

__device__ __forceinline__ uint16_t f32_to_f16_bits(float x) {
  _Float16 h = (_Float16)x;  // v_cvt_f16_f32: round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}

// Exact inverse normal CDF in FP64.  q = min(u, 1 - u); initial value from
// Abramowitz & Stegun 26.2.23 (Hastings' rational approximation in
// t = sqrt(-2 log q), |error| < 4.5e-4), then two Halley steps on
// f(z) = Phi(z) - q, f' = phi(z), f'' = -z phi(z):
//   z <- z - r / (1 + z r / 2),  r = f / phi(z).
// Phi(z) - q is formed as erf(z/sqrt2)/2 - (q - 1/2) when q >= 1/4 (the
// subtraction is exact there) and as erfc(-z/sqrt2)/2 - q otherwise.
// ITERS = 1 stops after one Halley step (|error| ~1e-10: a starting value).
template <int ITERS = 2>
__host__ __device__ __forceinline__ double exact_phi_inv(double u) {
  const bool upper = u > 0.5;
  const double q = upper ? 1.0 - u : u;
  const double t = sqrt(-2.0 * log(q));
  const double num = 2.515517 + t * (0.802853 + t * 0.010328);
  const double den = 1.0 + t * (1.432788 + t * (0.189269 + t * 0.001308));
  double z = num / den - t;
  const bool central = q >= 0.25;
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const double f = central ? 0.5 * erf(z * 0.70710678118654752440) - (q - 0.5)
                             : 0.5 * erfc(-z * 0.70710678118654752440) - q;
    const double pdf = 0.39894228040143267794 * exp(-0.5 * z * z);
    const double r = f / pdf;
    z = z - r / fma(0.5 * z, r, 1.0);
  }
  z = (q == 0.5) ? 0.0 : z;
  z = (q == 0.0) ? -__builtin_inf() : z;
  return upper ? -z : z;
}

}  // namespace aicdf
