// Streaming transforms U -> Z on gfx950: piecewise-constant lookup (Section
// 3.2, Code 1), dyadic piecewise polynomial (Section 3.3, Algorithm 1), the
// exact FP64 inverse (Section 3.1's role), the counter-based uniform fill and
// the HBM bandwidth probe (Section 3.4's "read and write" floor).
//
// The streaming transforms share one shape, chosen by measurement on MI355X:
// each thread moves four consecutive elements with one 16-byte non-temporal
// load and one 16-byte (8-byte for 16-bit outputs) non-temporal store,
// work-groups are a single 64-lane wave, and every work-group handles exactly
// one tile, so the launch holds the largest number of independent loads in
// flight.  Dyadic tables (<= 64 rows) live in registers, one row per lane,
// and are fetched with ds_bpermute: no LDS staging and no barrier.
#include "device_common.hpp"
#include "internal.hpp"

#include <algorithm>

using namespace aicdf;

namespace {

constexpr int kBlock = 256;
constexpr int kVec = 4;

enum OutKind { OUT_F64 = 0, OUT_F32 = 1, OUT_F16 = 2, OUT_BF16 = 3 };

template <int K> struct OutStore;
template <> struct OutStore<OUT_F64> { using T = double; };
template <> struct OutStore<OUT_F32> { using T = float; };
template <> struct OutStore<OUT_F16> { using T = uint16_t; };
template <> struct OutStore<OUT_BF16> { using T = uint16_t; };

template <int K> __device__ __forceinline__ typename OutStore<K>::T cvt_out(float x);
template <> __device__ __forceinline__ double cvt_out<OUT_F64>(float x) { return double(x); }
template <> __device__ __forceinline__ float cvt_out<OUT_F32>(float x) { return x; }
template <> __device__ __forceinline__ uint16_t cvt_out<OUT_F16>(float x) { return f32_to_f16_bits(x); }
template <> __device__ __forceinline__ uint16_t cvt_out<OUT_BF16>(float x) { return f32_to_bf16_bits(x); }

template <int K> __device__ __forceinline__ typename OutStore<K>::T cvt_out_d(double x);
template <> __device__ __forceinline__ double cvt_out_d<OUT_F64>(double x) { return x; }
template <> __device__ __forceinline__ float cvt_out_d<OUT_F32>(double x) { return float(x); }

__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
}
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
  const f64x2 b = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p) + 1);
  v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
}
__device__ __forceinline__ void store4(float* p, const float (&v)[4]) {
  __builtin_nontemporal_store(f32x4{v[0], v[1], v[2], v[3]}, reinterpret_cast<f32x4*>(p));
}
__device__ __forceinline__ void store4(double* p, const double (&v)[4]) {
  __builtin_nontemporal_store(f64x2{v[0], v[1]}, reinterpret_cast<f64x2*>(p));
  __builtin_nontemporal_store(f64x2{v[2], v[3]}, reinterpret_cast<f64x2*>(p) + 1);
}
__device__ __forceinline__ void store4(uint16_t* p, const uint16_t (&v)[4]) {
  __builtin_nontemporal_store(u16x4{v[0], v[1], v[2], v[3]}, reinterpret_cast<u16x4*>(p));
}

// ---------------------------------------------------------------- indices
// Row of a dyadic table (Algorithm 1, Table 1): the reflected u' lies in
// [2^-(e+1), 2^-e) for e = B - 1 - E(u'); the unsigned subtraction wraps for
// E > B - 1 (NaN, negative u') so that the cap sends those to the last row,
// as it does for u' = 0 and subnormals (E = 0).
__device__ __forceinline__ uint32_t dyadic_row_f32(float ur, uint32_t rows) {
  return min(126u - (__float_as_uint(ur) >> 23), rows - 1u);
}
__device__ __forceinline__ uint32_t dyadic_row_f64(double ur, uint32_t rows) {
  return min(1022u - uint32_t(__double_as_longlong(ur) >> 52), rows - 1u);
}
// Interval of a constant table (Code 1): floor(N u) clamped to [0, N-1];
// NaN maps to 0 (maxNum returns the non-NaN operand).
template <typename InT>
__device__ __forceinline__ uint32_t const_row(InT u, uint32_t n) {
  InT x = u * InT(n);  // exact: n is a power of two
  x = fmin(fmax(x, InT(0)), InT(n - 1));
  return uint32_t(x);
}

// ---------------------------------------------------------------- the ops
// Each op: `prep()` loads what every lane keeps in registers for the whole
// work-group (for dyadic tables: lane l holds row l, rows <= 64 = wave size),
// `eval(u, lane)` maps one uniform to the compute-precision result.  eval is
// always executed by all 64 lanes of a wave (the row fetch is a cross-lane
// ds_bpermute, which reads the source lane's register).

template <int DEG>
struct DyadicLane {
  float c[DEG + 1];
};

// The device table is padded to 64 rows of four floats, so every lane loads
// its row unconditionally, and only the DEG + 1 coefficients it needs (a
// wider load would leave dead registers that the compiler reuses only after
// waiting for this load, serialising it with the data stream).
template <int DEG>
__device__ __forceinline__ DyadicLane<DEG> dyadic_prep(const f32x4* tab, uint32_t) {
  const float* row = reinterpret_cast<const float*>(tab + __lane_id());
  DyadicLane<DEG> L;
  if constexpr (DEG == 0) {
    L.c[0] = row[0];
  } else if constexpr (DEG == 1) {
    const vec_t<float, 2> r = *reinterpret_cast<const vec_t<float, 2>*>(row);
    L.c[0] = r[0];
    L.c[1] = r[1];
  } else {
    const f32x4 r = *reinterpret_cast<const f32x4*>(row);
#pragma unroll
    for (int j = 0; j <= DEG; ++j) L.c[j] = r[j];
  }
  return L;
}

// coefficient j of row e, read from lane e
__device__ __forceinline__ float row_coef(uint32_t e, float mine) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(int(e << 2), __float_as_int(mine)));
}

// Dyadic table, FP32 input: Algorithm 1 in FP32.
template <int DEG>
struct DyadicF32 {
  const f32x4* tab;
  uint32_t rows;
  using In = float;
  using Acc = float;
  using Lane = DyadicLane<DEG>;
  __device__ Lane prep() const { return dyadic_prep<DEG>(tab, rows); }
  __device__ __forceinline__ float eval(float u, const Lane& L) const {
    const bool p = u < 0.5f;                      // predicate
    const float ur = p ? u : 1.0f - u;            // reflect (exact)
    const uint32_t e = dyadic_row_f32(ur, rows);  // exponent bits -> capped row
    const float s = ur * __uint_as_float((128u + e) << 23);  // u' 2^(e+1), exact
    float z = row_coef(e, L.c[DEG]);
    if (DEG == 0) z = fmaf(0.0f, s, z);  // NaN input stays NaN
#pragma unroll
    for (int j = DEG - 1; j >= 0; --j) z = fmaf(z, s, row_coef(e, L.c[j]));
    return p ? z : -z;
  }
};

// Dyadic table, FP64 input: index from the FP64 exponent, evaluation in FP64.
template <int DEG>
struct DyadicF64 {
  const f32x4* tab;
  uint32_t rows;
  using In = double;
  using Acc = double;
  using Lane = DyadicLane<DEG>;
  __device__ Lane prep() const { return dyadic_prep<DEG>(tab, rows); }
  __device__ __forceinline__ double eval(double u, const Lane& L) const {
    const bool p = u < 0.5;
    const double ur = p ? u : 1.0 - u;
    const uint32_t e = dyadic_row_f64(ur, rows);
    const double s = ur * __longlong_as_double((long long)(1024u + e) << 52);
    double z = double(row_coef(e, L.c[DEG]));
    if (DEG == 0) z = fma(0.0, s, z);  // NaN input stays NaN
#pragma unroll
    for (int j = DEG - 1; j >= 0; --j) z = fma(z, s, double(row_coef(e, L.c[j])));
    return p ? z : -z;
  }
};

// Geometric intervals with decay rate r (Theorem 2.5): lane l also holds the
// row threshold B_l (row e covers [B_e, B_(e-1)), the singular last row
// (0, B_(T-2))) and the scale 1/B_l of the local variable s = t / B_e.  The
// row coordinate x = log2(2t) / log2(r) puts row e at x in (e-1, e]; its
// FP32 estimate is within 1e-3 of the value the FP32 thresholds imply (log2
// error a few ulps of |log2 t| <= 127, |1/log2 r| <= 14), so ceil(x - 1/64)
// is the row or the one before it, and a single comparison with that row's
// lower threshold decides: the row is exact, the logarithm only narrows it.
template <int DEG>
struct GeometricLane {
  float c[DEG + 1];
  float thr, inv;
};

template <int DEG>
struct GeometricF32 {
  const f32x4* tab;  // 64 rows of four coefficients, then 64 thresholds, then 64 scales
  uint32_t rows;
  float inv_log2r;   // 1 / log2(r)
  using In = float;
  using Acc = float;
  using Lane = GeometricLane<DEG>;
  __device__ Lane prep() const {
    const DyadicLane<DEG> d = dyadic_prep<DEG>(tab, rows);
    Lane L;
#pragma unroll
    for (int j = 0; j <= DEG; ++j) L.c[j] = d.c[j];
    const float* extra = reinterpret_cast<const float*>(tab + 64);
    L.thr = extra[__lane_id()];
    L.inv = extra[64 + __lane_id()];
    return L;
  }
  __device__ __forceinline__ uint32_t row(float t, const Lane& L) const {
    // subnormal t: estimate from the least normal number (a NaN passes)
    const float t2 = 2.0f * t;
    const float x = __log2f(t2 < 0x1p-126f ? 0x1p-126f : t2) * inv_log2r;
    int e = int(fminf(fmaxf(ceilf(x - 0x1p-6f), 1.0f), float(rows - 1)));  // NaN -> 1
    const float lo = row_coef(uint32_t(e), L.thr);  // lower bound of row e
    if (e < int(rows) - 1 && t < lo) ++e;
    return t >= 0.5f ? 0u : uint32_t(e);
  }
  __device__ __forceinline__ float eval(float u, const Lane& L) const {
    const bool p = u < 0.5f;
    const float t = p ? u : 1.0f - u;
    const uint32_t e = row(t, L);
    const float s = t * row_coef(e, L.inv);
    float z = row_coef(e, L.c[DEG]);
    if (DEG == 0) z = fmaf(0.0f, s, z);
#pragma unroll
    for (int j = DEG - 1; j >= 0; --j) z = fmaf(z, s, row_coef(e, L.c[j]));
    return p ? z : -z;
  }
};

struct NoLane {};

// Constant table with FP32 entries: gathered through the vector L1/L2 (the
// 4 KiB table of 1024 intervals stays cache resident).
template <typename InT>
struct ConstF32 {
  const float* tab;
  uint32_t n;
  using In = InT;
  using Acc = InT;  // the FP32 constant, widened for FP64 input
  using Lane = NoLane;
  __device__ Lane prep() const { return {}; }
  __device__ __forceinline__ InT eval(InT u, const Lane&) const { return InT(__ldg(tab + const_row(u, n))); }
};

// Constant table with FP64 entries (FP64 input only).
struct ConstF64 {
  const double* tab;
  uint32_t n;
  using In = double;
  using Acc = double;
  using Lane = NoLane;
  __device__ Lane prep() const { return {}; }
  __device__ __forceinline__ double eval(double u, const Lane&) const { return __ldg(tab + const_row(u, n)); }
};

// Exact inverse normal (FP64 arithmetic for either input precision).
template <typename InT>
struct Exact {
  using In = InT;
  using Acc = double;
  using Lane = NoLane;
  __device__ Lane prep() const { return {}; }
  __device__ __forceinline__ double eval(InT u, const Lane&) const { return exact_phi_inv(double(u)); }
};

template <int K, typename Acc> struct Cvt;
template <int K> struct Cvt<K, float> {
  __device__ static typename OutStore<K>::T go(float x) { return cvt_out<K>(x); }
};
template <int K> struct Cvt<K, double> {
  __device__ static typename OutStore<K>::T go(double x) { return cvt_out_d<K>(x); }
};

// One thread transforms four consecutive elements; one 64-lane wave per
// work-group; one tile per work-group (no grid-stride loop), which keeps the
// most independent loads in flight.  `first` offsets the launch within the
// array (launches are split at 2^30 threads).
constexpr int kStreamBlock = 64;

template <class Op, int OUTK>
__global__ __launch_bounds__(kStreamBlock) void transform_kernel(const typename Op::In* __restrict__ u,
                                                                 typename OutStore<OUTK>::T* __restrict__ z,
                                                                 size_t n, size_t first, Op op, int vec_ok) {
  using InT = typename Op::In;
  using OutT = typename OutStore<OUTK>::T;
  using Acc = typename Op::Acc;
  const size_t i0 = first + (size_t(blockIdx.x) * kStreamBlock + threadIdx.x) * kVec;
  const size_t blk_end = first + (size_t(blockIdx.x) + 1) * kStreamBlock * kVec;
  if (vec_ok && blk_end <= n) {  // uniform per work-group
    InT x[4];
    load4(u + i0, x);  // the data load is issued first
    const typename Op::Lane lane = op.prep();
    OutT y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = Cvt<OUTK, Acc>::go(op.eval(x[k], lane));
    store4(z + i0, y);
  } else {
    const typename Op::Lane lane = op.prep();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const size_t i = i0 + k;
      const InT x = i < n ? u[i] : InT(0.5);
      const OutT y = Cvt<OUTK, Acc>::go(op.eval(x, lane));
      if (i < n) z[i] = y;
    }
  }
}

int g_num_cus = 0;

int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
      g_num_cus = c;
    else
      g_num_cus = 256;
  }
  return g_num_cus;
}

template <class Op, int OUTK>
aicdf_status launch_transform(const void* u, void* z, size_t n, const Op& op, hipStream_t stream) {
  using InT = typename Op::In;
  using OutT = typename OutStore<OUTK>::T;
  const int vec_ok = aligned(u, kVec * sizeof(InT)) && aligned(z, kVec * sizeof(OutT));
  const size_t per_block = size_t(kStreamBlock) * kVec;
  const size_t max_blocks = size_t(1) << 24;  // 2^30 threads per launch
  for (size_t first = 0; first < n; first += max_blocks * per_block) {
    const size_t rem = n - first;
    const size_t blocks = std::min(max_blocks, (rem + per_block - 1) / per_block);
    hipLaunchKernelGGL((transform_kernel<Op, OUTK>), dim3(unsigned(blocks)), dim3(kStreamBlock), 0, stream,
                       static_cast<const InT*>(u), static_cast<OutT*>(z), n, first, op, vec_ok);
  }
  AICDF_HIP(hipGetLastError());
  return ok();
}

template <class Op>
aicdf_status dispatch_out(const void* u, void* z, aicdf_dtype z_t, size_t n, const Op& op, hipStream_t s) {
  using Acc = typename Op::Acc;
  if constexpr (sizeof(Acc) == 4) {
    switch (z_t) {
      case AICDF_F32: return launch_transform<Op, OUT_F32>(u, z, n, op, s);
      case AICDF_F16: return launch_transform<Op, OUT_F16>(u, z, n, op, s);
      case AICDF_BF16: return launch_transform<Op, OUT_BF16>(u, z, n, op, s);
      default: break;
    }
  } else {
    switch (z_t) {
      case AICDF_F32: return launch_transform<Op, OUT_F32>(u, z, n, op, s);
      case AICDF_F64: return launch_transform<Op, OUT_F64>(u, z, n, op, s);
      default: break;
    }
  }
  return fail(AICDF_EDTYPE, "unsupported output dtype %d for this input dtype", int(z_t));
}

aicdf_status check_io(size_t n, const void* u, aicdf_dtype u_t, const void* z, aicdf_dtype z_t) {
  if (!dtype_valid(u_t) || !dtype_valid(z_t)) return fail(AICDF_EDTYPE, "invalid dtype");
  if (n == 0) return AICDF_OK;
  if (!u || !z) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (overlaps(u, n * dtype_size(u_t), z, n * dtype_size(z_t)))
    return fail(AICDF_EALIAS, "input and output ranges overlap");
  return AICDF_OK;
}

aicdf_status check_table_device(const aicdf_table* t) {
  int dev = 0;
  AICDF_HIP(hipGetDevice(&dev));
  if (dev != t->device) return fail(AICDF_EINVAL, "table lives on device %d, current device is %d", t->device, dev);
  return AICDF_OK;
}

}  // namespace

extern "C" aicdf_status approx_icdf_linear(const aicdf_table* t, size_t n, const void* u,
                                           aicdf_dtype u_t, void* z, aicdf_dtype z_t, void* stream) {
  if (!t) return fail(AICDF_EINVAL, "table is NULL");
  if (t->kind != 1 && t->kind != 2)
    return fail(AICDF_EINVAL, "approx_icdf_linear needs a dyadic or geometric table");
  aicdf_status st = check_io(n, u, u_t, z, z_t);
  if (st != AICDF_OK || n == 0) return st == AICDF_OK ? ok() : st;
  if ((st = check_table_device(t)) != AICDF_OK) return st;
  auto s = static_cast<hipStream_t>(stream);
  const auto* tab = static_cast<const f32x4*>(t->dev);
  const int deg = int(t->cols) - 1;
  if (t->kind == 2) {
    if (u_t != AICDF_F32) return fail(AICDF_EDTYPE, "geometric tables take F32 input");
    const float il = float(1.0 / std::log2(t->r));
    switch (deg) {
      case 0: return dispatch_out(u, z, z_t, n, GeometricF32<0>{tab, t->rows, il}, s);
      case 1: return dispatch_out(u, z, z_t, n, GeometricF32<1>{tab, t->rows, il}, s);
      case 2: return dispatch_out(u, z, z_t, n, GeometricF32<2>{tab, t->rows, il}, s);
      default: return dispatch_out(u, z, z_t, n, GeometricF32<3>{tab, t->rows, il}, s);
    }
  }
  if (u_t == AICDF_F32) {
    switch (deg) {
      case 0: return dispatch_out(u, z, z_t, n, DyadicF32<0>{tab, t->rows}, s);
      case 1: return dispatch_out(u, z, z_t, n, DyadicF32<1>{tab, t->rows}, s);
      case 2: return dispatch_out(u, z, z_t, n, DyadicF32<2>{tab, t->rows}, s);
      default: return dispatch_out(u, z, z_t, n, DyadicF32<3>{tab, t->rows}, s);
    }
  }
  if (u_t == AICDF_F64) {
    switch (deg) {
      case 0: return dispatch_out(u, z, z_t, n, DyadicF64<0>{tab, t->rows}, s);
      case 1: return dispatch_out(u, z, z_t, n, DyadicF64<1>{tab, t->rows}, s);
      case 2: return dispatch_out(u, z, z_t, n, DyadicF64<2>{tab, t->rows}, s);
      default: return dispatch_out(u, z, z_t, n, DyadicF64<3>{tab, t->rows}, s);
    }
  }
  return fail(AICDF_EDTYPE, "input dtype must be F32 or F64");
}

extern "C" aicdf_status approx_icdf_const(const aicdf_table* t, size_t n, const void* u,
                                          aicdf_dtype u_t, void* z, aicdf_dtype z_t, void* stream) {
  if (!t) return fail(AICDF_EINVAL, "table is NULL");
  if (t->kind != 0) return fail(AICDF_EINVAL, "approx_icdf_const needs a constant table");
  aicdf_status st = check_io(n, u, u_t, z, z_t);
  if (st != AICDF_OK || n == 0) return st == AICDF_OK ? ok() : st;
  if ((st = check_table_device(t)) != AICDF_OK) return st;
  auto s = static_cast<hipStream_t>(stream);
  if (t->coef_t == AICDF_F64) {
    if (u_t != AICDF_F64) return fail(AICDF_EDTYPE, "an F64 constant table needs F64 input");
    return dispatch_out(u, z, z_t, n, ConstF64{static_cast<const double*>(t->dev), t->rows}, s);
  }
  const auto* tab = static_cast<const float*>(t->dev);
  if (u_t == AICDF_F32) return dispatch_out(u, z, z_t, n, ConstF32<float>{tab, t->rows}, s);
  // FP64 input with FP32 constants: the index is taken in FP64 and the FP32
  // constant is widened (exact) before the output conversion
  if (u_t == AICDF_F64) return dispatch_out(u, z, z_t, n, ConstF32<double>{tab, t->rows}, s);
  return fail(AICDF_EDTYPE, "input dtype must be F32 or F64");
}

namespace {
template <typename InT>
__global__ __launch_bounds__(kBlock) void index_kernel(const InT* __restrict__ u, uint32_t* __restrict__ idx,
                                                       size_t n, int dyadic, uint32_t rows) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += size_t(gridDim.x) * kBlock) {
    const InT x = u[i];
    uint32_t r;
    if (dyadic) {
      const InT ur = x < InT(0.5) ? x : InT(1) - x;
      if constexpr (sizeof(InT) == 4)
        r = dyadic_row_f32(ur, rows);
      else
        r = dyadic_row_f64(ur, rows);
    } else {
      r = const_row(x, rows);
    }
    idx[i] = r;
  }
}
}  // namespace

namespace {
// Rows of a geometric table, one wave per 64 consecutive inputs (all lanes
// take part in the cross-lane threshold reads; lanes past n use t = 1/4).
__global__ __launch_bounds__(kStreamBlock) void geometric_index_kernel(const float* __restrict__ u,
                                                                       uint32_t* __restrict__ idx, size_t n,
                                                                       GeometricF32<0> op) {
  const GeometricLane<0> L = op.prep();
  const size_t i = size_t(blockIdx.x) * kStreamBlock + threadIdx.x;
  const float x = i < n ? u[i] : 0.25f;
  const float t = x < 0.5f ? x : 1.0f - x;
  const uint32_t r = op.row(t, L);
  if (i < n) idx[i] = r;
}
}  // namespace

extern "C" aicdf_status approx_icdf_index(const aicdf_table* t, size_t n, const void* u, aicdf_dtype u_t,
                                          uint32_t* idx, void* stream) {
  if (!t) return fail(AICDF_EINVAL, "table is NULL");
  aicdf_status st = check_io(n, u, u_t, idx, AICDF_F32);
  if (st != AICDF_OK || n == 0) return st == AICDF_OK ? ok() : st;
  if (u_t != AICDF_F32 && u_t != AICDF_F64) return fail(AICDF_EDTYPE, "input dtype must be F32 or F64");
  if ((st = check_table_device(t)) != AICDF_OK) return st;
  if (t->kind == 2) {
    if (u_t != AICDF_F32) return fail(AICDF_EDTYPE, "geometric tables take F32 input");
    const GeometricF32<0> op{static_cast<const f32x4*>(t->dev), t->rows, float(1.0 / std::log2(t->r))};
    const size_t blocks = (n + kStreamBlock - 1) / kStreamBlock;
    for (size_t b0 = 0; b0 < blocks; b0 += size_t(1) << 30) {
      const size_t nb = std::min(blocks - b0, size_t(1) << 30);
      const size_t first = b0 * kStreamBlock;
      hipLaunchKernelGGL(geometric_index_kernel, dim3(unsigned(nb)), dim3(kStreamBlock), 0,
                         static_cast<hipStream_t>(stream), static_cast<const float*>(u) + first, idx + first,
                         n - first, op);
    }
    AICDF_HIP(hipGetLastError());
    return ok();
  }
  const size_t need = (n + kBlock - 1) / kBlock;
  const size_t maxg = size_t(num_cus()) * 16;
  const unsigned grid = unsigned(need < maxg ? need : maxg);
  auto s = static_cast<hipStream_t>(stream);
  if (u_t == AICDF_F32)
    hipLaunchKernelGGL(index_kernel<float>, dim3(grid), dim3(kBlock), 0, s, static_cast<const float*>(u), idx, n,
                       t->kind, t->rows);
  else
    hipLaunchKernelGGL(index_kernel<double>, dim3(grid), dim3(kBlock), 0, s, static_cast<const double*>(u), idx, n,
                       t->kind, t->rows);
  AICDF_HIP(hipGetLastError());
  return ok();
}

extern "C" aicdf_status exact_icdf(size_t n, const void* u, aicdf_dtype u_t, void* z, aicdf_dtype z_t,
                                   void* stream) {
  aicdf_status st = check_io(n, u, u_t, z, z_t);
  if (st != AICDF_OK || n == 0) return st == AICDF_OK ? ok() : st;
  auto s = static_cast<hipStream_t>(stream);
  if (u_t == AICDF_F64) return dispatch_out(u, z, z_t, n, Exact<double>{}, s);
  if (u_t == AICDF_F32) return dispatch_out(u, z, z_t, n, Exact<float>{}, s);
  return fail(AICDF_EDTYPE, "input dtype must be F32 or F64");
}

// ------------------------------------------------------------------ uniforms
namespace {

// One Philox block (four 32-bit words) per thread, one tile per work-group.
__global__ __launch_bounds__(kStreamBlock) void uniform_f32_kernel(float* __restrict__ u, size_t n, uint64_t offset,
                                                                   uint32_t k0, uint32_t k1, uint32_t s0, uint32_t s1,
                                                                   uint64_t first_block, uint64_t nblocks) {
  const uint64_t t = uint64_t(blockIdx.x) * kStreamBlock + threadIdx.x;
  if (t >= nblocks) return;
  const uint64_t b = first_block + t;
  const u32x4 w = philox4x32_10(uint32_t(b), uint32_t(b >> 32), s0, s1, k0, k1);
  const uint64_t g0 = b * 4;  // first word of this block
  if (g0 >= offset && g0 + 4 <= offset + n && ((g0 - offset) & 3) == 0 && (reinterpret_cast<uintptr_t>(u) & 15) == 0) {
    __builtin_nontemporal_store(f32x4{u24_from_word(w[0]), u24_from_word(w[1]), u24_from_word(w[2]), u24_from_word(w[3])},
                                reinterpret_cast<f32x4*>(u + (g0 - offset)));
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t g = g0 + j;
      if (g >= offset && g < offset + n) u[g - offset] = u24_from_word(w[j]);
    }
  }
}

__global__ __launch_bounds__(kStreamBlock) void uniform_f64_kernel(double* __restrict__ u, size_t n, uint64_t offset,
                                                                   uint32_t k0, uint32_t k1, uint32_t s0, uint32_t s1,
                                                                   uint64_t first_block, uint64_t nblocks) {
  const uint64_t t = uint64_t(blockIdx.x) * kStreamBlock + threadIdx.x;
  if (t >= nblocks) return;
  const uint64_t b = first_block + t;
  const u32x4 w = philox4x32_10(uint32_t(b), uint32_t(b >> 32), s0, s1, k0, k1);
  const uint64_t g0 = b * 2;
  const double a = u53_from_words(w[0], w[1]);
  const double c = u53_from_words(w[2], w[3]);
  if (g0 >= offset && g0 + 2 <= offset + n && ((g0 - offset) & 1) == 0 && (reinterpret_cast<uintptr_t>(u) & 15) == 0) {
    __builtin_nontemporal_store(f64x2{a, c}, reinterpret_cast<f64x2*>(u + (g0 - offset)));
  } else {
    if (g0 >= offset && g0 < offset + n) u[g0 - offset] = a;
    if (g0 + 1 >= offset && g0 + 1 < offset + n) u[g0 + 1 - offset] = c;
  }
}

}  // namespace

extern "C" aicdf_status aicdf_uniform_fill(uint64_t seed, uint64_t stream_id, uint64_t offset, size_t n,
                                           void* u, aicdf_dtype u_t, void* stream) {
  if (u_t != AICDF_F32 && u_t != AICDF_F64) return fail(AICDF_EDTYPE, "uniforms are F32 or F64");
  if (n == 0) return ok();
  if (!u) return fail(AICDF_EINVAL, "NULL buffer with n = %zu", n);
  if (offset + n < offset) return fail(AICDF_ERANGE, "offset + n overflows");
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  const uint32_t s0 = uint32_t(stream_id), s1 = uint32_t(stream_id >> 32);
  const int per = (u_t == AICDF_F32) ? 4 : 2;
  const uint64_t first = offset / per, last = (offset + n - 1) / per;
  const uint64_t total = last - first + 1;
  auto s = static_cast<hipStream_t>(stream);
  const uint64_t max_threads = uint64_t(1) << 30;
  for (uint64_t done = 0; done < total; done += max_threads) {
    const uint64_t cnt = std::min(max_threads, total - done);
    const unsigned grid = unsigned((cnt + kStreamBlock - 1) / kStreamBlock);
    if (u_t == AICDF_F32)
      hipLaunchKernelGGL(uniform_f32_kernel, dim3(grid), dim3(kStreamBlock), 0, s, static_cast<float*>(u), n, offset,
                         k0, k1, s0, s1, first + done, cnt);
    else
      hipLaunchKernelGGL(uniform_f64_kernel, dim3(grid), dim3(kStreamBlock), 0, s, static_cast<double*>(u), n, offset,
                         k0, k1, s0, s1, first + done, cnt);
  }
  AICDF_HIP(hipGetLastError());
  return ok();
}

// ------------------------------------------------------------------ bandwidth
namespace {

// One 16-byte vector per thread, one tile per 64-lane work-group (the shape
// of the streaming transforms).  Mode 1 folds what it reads into a value that
// is stored only if it equals an impossible sentinel, so the loads stay live.
template <int MODE>
__global__ __launch_bounds__(kStreamBlock) void bw_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                          size_t n16, size_t first) {
  const size_t i = first + size_t(blockIdx.x) * kStreamBlock + threadIdx.x;
  if (i >= n16) return;
  if (MODE == 2) {
    __builtin_nontemporal_store(f32x4{float(i), 0.f, 0.f, 0.f}, dst + i);
    return;
  }
  const f32x4 v = __builtin_nontemporal_load(src + i);
  if (MODE == 0) {
    __builtin_nontemporal_store(v, dst + i);
  } else {
    const float a = v[0] + v[1] + v[2] + v[3];
    if (a == -1.2345e-38f) dst[0] = v;
  }
}

}  // namespace

extern "C" aicdf_status aicdf_bw_probe(int32_t mode, size_t n_bytes, const void* src, void* dst, void* stream) {
  if (mode < 0 || mode > 2) return fail(AICDF_EINVAL, "mode must be 0 (copy), 1 (read) or 2 (write)");
  if (n_bytes == 0) return ok();
  if (n_bytes % 16) return fail(AICDF_EINVAL, "n_bytes must be a multiple of 16");
  if ((mode != 2 && (!src || !aligned(src, 16))) || !dst || !aligned(dst, 16))
    return fail(AICDF_EINVAL, "buffers must be non-NULL and 16-byte aligned");
  const size_t n16 = n_bytes / 16;
  if (mode == 0 && overlaps(src, n_bytes, dst, n_bytes)) return fail(AICDF_EALIAS, "src and dst overlap");
  auto s = static_cast<hipStream_t>(stream);
  auto* d = static_cast<f32x4*>(dst);
  const auto* a = static_cast<const f32x4*>(src);
  const size_t max_threads = size_t(1) << 30;
  for (size_t first = 0; first < n16; first += max_threads) {
    const size_t cnt = std::min(max_threads, n16 - first);
    const unsigned grid = unsigned((cnt + kStreamBlock - 1) / kStreamBlock);
    if (mode == 0)
      hipLaunchKernelGGL(bw_kernel<0>, dim3(grid), dim3(kStreamBlock), 0, s, a, d, n16, first);
    else if (mode == 1)
      hipLaunchKernelGGL(bw_kernel<1>, dim3(grid), dim3(kStreamBlock), 0, s, a, d, n16, first);
    else
      hipLaunchKernelGGL(bw_kernel<2>, dim3(grid), dim3(kStreamBlock), 0, s, a, d, n16, first);
  }
  AICDF_HIP(hipGetLastError());
  return ok();
}
