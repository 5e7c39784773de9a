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
    // each 32 x 32 -> 64-bit product in one instruction (v_mad_u64_u32)
    const uint64_t p0 = uint64_t(c0) * 0xD2511F53u, p1 = uint64_t(c2) * 0xCD9E8D57u;
    const uint32_t lo0 = uint32_t(p0), hi0 = uint32_t(p0 >> 32);
    const uint32_t lo1 = uint32_t(p1), hi1 = uint32_t(p1 >> 32);
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

// Exact inverse normal CDF in FP64: Wichura's algorithm AS 241 (PPND16,
// Applied Statistics 37 (1988) 477-484).  With q = u - 1/2:
//   |q| <= 0.425   z = q A(r) / B(r),  r = 0.180625 - q^2
//   otherwise      s = sqrt(-log(min(u, 1 - u)));  z = +-C(s - 1.6) / D(s - 1.6)
//                  for s <= 5, +-E(s - 5) / F(s - 5) beyond (sign of q)
// with A..F polynomials of degree 7 (published coefficients).  Relative
// error about 1e-16 by design, below 1e-15 measured against 50-digit roots;
// a few FMAs and one division in the centre, one log and one sqrt more in
// the tails (no iteration).  u = 0 and u = 1 give -inf and +inf.
// The coefficients of AS 241 (PPND16): numerator and denominator of the
// central region (A, B), the middle tail (C, D) and the far tail (E, F).
constexpr double kAs241A[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2, 1.9715909503065514427e+3,
                               1.3731693765509461125e+4, 4.5921953931549871457e+4, 6.7265770927008700853e+4,
                               3.3430575583588128105e+4, 2.5090809287301226727e+3};
constexpr double kAs241B[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2, 5.3941960214247511077e+3,
                               2.1213794301586595867e+4, 3.9307895800092710610e+4, 2.8729085735721942674e+4,
                               5.2264952788528545610e+3};
constexpr double kAs241C[8] = {1.42343711074968357734e0, 4.63033784615654529590e0, 5.76949722146069140550e0,
                               3.64784832476320460504e0, 1.27045825245236838258e0, 2.41780725177450611770e-1,
                               2.27238449892691845833e-2, 7.74545014278341407640e-4};
constexpr double kAs241D[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0, 6.89767334985100004550e-1,
                               1.48103976427480074590e-1, 1.51986665636164571966e-2, 5.47593808499534494600e-4,
                               1.05075007164441684324e-9};
constexpr double kAs241E[8] = {6.65790464350110377720e0, 5.46378491116411436990e0, 1.78482653991729133580e0,
                               2.96560571828504891230e-1, 2.65321895265761230930e-2, 1.24266094738807843860e-3,
                               2.71155556874348757815e-5, 2.01033439929228813265e-7};
constexpr double kAs241F[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1, 1.48753612908506148525e-2,
                               7.86869131145613259100e-4, 1.84631831751005468180e-5, 1.42151175831644588870e-7,
                               2.04426310338993978564e-15};

__host__ __device__ __forceinline__ double phi_inv_poly7(const double (&c)[8], double x) {
  double s = c[7];
#pragma unroll
  for (int k = 6; k >= 0; --k) s = fma(s, x, c[k]);
  return s;
}

__host__ __device__ __forceinline__ double exact_phi_inv(double u) {
  const auto& A = kAs241A;
  const auto& B = kAs241B;
  const auto& C = kAs241C;
  const auto& D = kAs241D;
  const auto& E = kAs241E;
  const auto& F = kAs241F;
  const double q = u - 0.5;
  if (fabs(q) <= 0.425) {
    const double r = fma(-q, q, 0.180625);
    return q * phi_inv_poly7(A, r) / phi_inv_poly7(B, r);
  }
  if (u == 0.0) return -__builtin_inf();
  if (u == 1.0) return __builtin_inf();
  const double s = sqrt(-log(fmin(u, 1.0 - u)));
  const bool mid = s <= 5.0;
  const double x = s - (mid ? 1.6 : 5.0);
  const double z = mid ? phi_inv_poly7(C, x) / phi_inv_poly7(D, x) : phi_inv_poly7(E, x) / phi_inv_poly7(F, x);
  return q < 0.0 ? -z : z;
}

// Phi^-1 in FP32 for an approximation whose own error is far larger (the
// Sankaran comparator): the rational functions of AS 241 evaluated in FP32
// arithmetic (relative error a few FP32 ulps).  u = 0 and u = 1 give -inf and
// +inf.
__device__ __forceinline__ float phi_inv_poly7f(const double (&c)[8], float x) {
  float s = float(c[7]);
#pragma unroll
  for (int k = 6; k >= 0; --k) s = fmaf(s, x, float(c[k]));
  return s;
}

__device__ __forceinline__ float approx_phi_inv_f32(float u) {
  const float q = u - 0.5f;
  if (fabsf(q) <= 0.425f) {
    const float r = fmaf(-q, q, 0.180625f);
    return q * phi_inv_poly7f(kAs241A, r) / phi_inv_poly7f(kAs241B, r);
  }
  if (u == 0.0f) return -__builtin_inff();
  if (u == 1.0f) return __builtin_inff();
  const float s = sqrtf(-logf(fminf(u, 1.0f - u)));
  const bool mid = s <= 5.0f;
  const float x = s - (mid ? 1.6f : 5.0f);
  const float z = mid ? phi_inv_poly7f(kAs241C, x) / phi_inv_poly7f(kAs241D, x)
                      : phi_inv_poly7f(kAs241E, x) / phi_inv_poly7f(kAs241F, x);
  return q < 0.0f ? -z : z;
}

}  // namespace aicdf
