// Internal host-side helpers of libaicdf: status/error plumbing, the table
// handle, and small argument checks.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/aicdf.h"

namespace aicdf {

// Sets the thread-local error text and returns `code`.
aicdf_status fail(aicdf_status code, const char* fmt, ...);
// Clears the thread-local error text and returns AICDF_OK.
aicdf_status ok();

#define AICDF_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::aicdf::fail(AICDF_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

inline size_t dtype_size(aicdf_dtype t) {
  switch (t) {
    case AICDF_F64: return 8;
    case AICDF_F32: return 4;
    case AICDF_F16: return 2;
    case AICDF_BF16: return 2;
  }
  return 0;
}

inline bool dtype_valid(int t) { return t >= AICDF_F64 && t <= AICDF_BF16; }

// True when [a, a+na) and [b, b+nb) share a byte.
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Host FP64 builders (host_tables.cpp).
double host_Phi(double z);
double host_phi(double z);
double host_Phi_inv(double u);
std::vector<double> build_const_table(uint32_t n, int construction);
std::vector<double> build_dyadic_table(uint32_t n_entries, uint32_t degree);
std::vector<double> geometric_thresholds(double r, uint32_t n_entries);
std::vector<double> build_geometric_table(double r, uint32_t n_entries, uint32_t degree);
double round_to_dtype(double x, aicdf_dtype t);
// n-point Gauss-Legendre rule on [-1, 1]; small dense solve (n <= 4, A and b overwritten, b := A^-1 b).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void solve_small(int n, double* A, double* b);

// Surrogate internals used by the CIR level (surrogate.hip).
const float* surrogate_params(const aicdf_surrogate* s);
const uint16_t* surrogate_w2b(const aicdf_surrogate* s);
const float* surrogate_wtab(const aicdf_surrogate* s);
void surrogate_range(const aicdf_surrogate* s, double* nu, double* lo, double* hi, int* dev);

// Chi-squared table internals used by the CIR level (chi2_table.hip).
struct Chi2Info {
  double nu;
  uint32_t degree, n_knots, n_intervals;
  int device;
  const void* dev_rows;  // n_knots * 2 * n_intervals FP32 rows of four
};
Chi2Info chi2_info(const aicdf_chi2_table* t);

}  // namespace aicdf

// A coefficient table: host FP64 copy of the stored (dtype-rounded) values
// and a device copy.  Dyadic tables are stored on the device as 64 FP32 rows
// of four (c0..c3; rows and columns beyond the table are zero); geometric
// tables likewise, followed by 64 FP32 row thresholds B_e and 64 FP32 scales
// 1/B_e (zero beyond the table); constant
// tables as FP32, or FP64 when coef_t is F64.  FP16/BF16 coefficients are exactly representable in FP32, so the
// device copy holds the rounded values without further error.
struct aicdf_table {
  int kind;  // 0 constant, 1 dyadic, 2 geometric (decay rate r)
  uint32_t rows, cols;
  int construction;
  aicdf_dtype coef_t;
  int device;
  std::vector<double> host;  // rows x cols, rounded to coef_t
  void* dev;                 // device copy (see above)
  size_t dev_bytes;
  double r;                  // geometric tables: decay rate
};
