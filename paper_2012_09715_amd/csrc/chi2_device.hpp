// Device evaluation of the piecewise-polynomial approximation of the
// non-central chi-squared inverse CDF (Section 5.1):
//   C~^-1(U; lambda) = lambda + nu + 2 sqrt(lambda + nu) P~(U; y),
//   y = nu / (lambda + nu),
// P~ interpolated linearly in sqrt(y) between the two neighbouring knots
// sqrt(y_i) = i / (K - 1), each knot holding two dyadic tables (U <= 1/2 in
// t = U, U > 1/2 in t = 1 - U).  Interval k = 1..n-1 of a half covers
// t in [2^-(k+1), 2^-k), interval n the singular (0, 2^-n); a row holds the
// coefficients of the interval's polynomial in s = t 2^(k+1).
//
// Table layout (FP32 rows of four, c0..c3, unused degrees zero):
//   row ((i * 2 + half) * n + (k - 1)).
#pragma once

#include "device_common.hpp"

namespace aicdf {

struct Chi2Geom {
  float nu, sqrt_nu, kmax;  // kmax = K - 1
  uint32_t seg_max;         // K - 2, the last knot segment
  uint32_t n_int;           // intervals per half
};

template <int DEG>
__device__ __forceinline__ float chi2_horner(const f32x4* __restrict__ row, float s) {
  if constexpr (DEG == 1) {
    const vec_t<float, 2> c = *reinterpret_cast<const vec_t<float, 2>*>(row);
    return fmaf(c[1], s, c[0]);
  } else {
    const f32x4 c = *row;
    return fmaf(fmaf(fmaf(c[3], s, c[2]), s, c[1]), s, c[0]);
  }
}

// x~ for one (u, lambda) in FP32.  Any input stays in bounds of the table:
// the interval index is capped by unsigned arithmetic on the exponent bits of
// t (t = 1/2 -> interval 1; t = 0, subnormal, negative or NaN -> the singular
// interval) and the knot coordinate is clamped to [0, K - 1].  lambda < 0 or
// NaN gives NaN.
template <int DEG>
__device__ __forceinline__ float chi2_approx_x(float u, float lam, const f32x4* __restrict__ tab, const Chi2Geom& g) {
  const float s = lam + g.nu;
  const float r = rsqrtf(s);
  const float fq = fminf(fmaxf(g.sqrt_nu * r * g.kmax, 0.0f), g.kmax);
  const uint32_t i = min(uint32_t(fq), g.seg_max);
  const float th = fq - float(i);
  const bool up = u > 0.5f;
  const float t = up ? 1.0f - u : u;
  const uint32_t k = min(max(126u - (__float_as_uint(t) >> 23), 1u), g.n_int);
  const float sl = t * __uint_as_float((128u + k) << 23);  // t 2^(k+1)
  const f32x4* row0 = tab + (i * 2u + (up ? 1u : 0u)) * g.n_int + (k - 1u);
  const f32x4* row1 = row0 + 2u * g.n_int;
  const float p0 = chi2_horner<DEG>(row0, sl);
  const float p1 = chi2_horner<DEG>(row1, sl);
  const float P = fmaf(th, p1 - p0, p0);
  const float x = fmaf(2.0f * s * r, P, s);  // 2 sqrt(s) = 2 s / sqrt(s)
  return lam >= 0.0f ? x : __builtin_nanf("");
}

// The Sankaran approximation, Section 5.1's comparator (Table 6d), in FP32
// (the normal quantile too: AS 241 in FP32, far below the approximation's own
// error): with k = nu,
//   c1 = 1 - (2/3)(k+lambda)(k+3 lambda)/(k+2 lambda)^2,
//   c2 = (k+2 lambda)/(k+lambda)^2,  c3 = (c1-1)(1-3 c1),
//   B  = 1 + c1 c2 (c1 - 1 + (2-c1) c2 c3/2) + c1 sqrt(2 c2)(1 + c2 c3/2) Phi^-1(u),
//   x~ = (k+lambda) max(B, 0)^(1/c1).
// The square root of the Gaussian term is read as sqrt(2 c2) and B is clamped
// at 0 (both fixed by Table 6d).  lambda < 0 or NaN gives NaN.
__device__ __forceinline__ float sankaran_x(float u, float lam, float nu) {
  const float kl = nu + lam, k2l = fmaf(2.0f, lam, nu), k3l = fmaf(3.0f, lam, nu);
  const float c1 = 1.0f - (2.0f / 3.0f) * kl * k3l / (k2l * k2l);
  const float c2 = k2l / (kl * kl);
  const float c3 = (c1 - 1.0f) * (1.0f - 3.0f * c1);
  const float z = approx_phi_inv_f32(u);
  const float a = fmaf(0.5f * (2.0f - c1) * c2, c3, c1 - 1.0f);
  const float g = c1 * sqrtf(2.0f * c2) * fmaf(0.5f * c2, c3, 1.0f);
  const float B = fmaf(g, z, fmaf(c1 * c2, a, 1.0f));
  const float x = kl * powf(fmaxf(B, 0.0f), 1.0f / c1);
  return lam >= 0.0f ? x : __builtin_nanf("");
}

}  // namespace aicdf
