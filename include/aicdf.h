/*
 * aicdf.h -- C ABI of libaicdf.so: approximate inverse-CDF random variables
 * and nested multilevel Monte Carlo levels on AMD Instinct MI355X (gfx950).
 *
 * Method: Giles & Sheridan-Methven, "Approximating inverse cumulative
 * distribution functions to produce approximate random variables"
 * (arXiv:2012.09715).  Section numbers below refer to that paper.
 *
 * Conventions (all entry points)
 *  - Pointers named "device" are HIP device pointers on the current device;
 *    pointers named "host" are host memory.  The caller owns every buffer it
 *    passes; the library never frees caller memory.
 *  - Opaque handles (aicdf_table, aicdf_chi2_table, aicdf_surrogate) are library-owned and are
 *    released with their destroy call; destroy(NULL) is a no-op.  A handle is
 *    bound to the device that was current when it was created.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Transform calls only enqueue work and return; the MLMC level calls (not
 *    their _async forms) and the calls returning host results synchronise
 *    `stream` before returning.
 *  - Errors are reported only through the status code; aicdf_last_error()
 *    returns a thread-local text for the last failing call.  No call prints,
 *    throws across the ABI or aborts.
 *  - n == 0 is a successful no-op.  A NULL data pointer with n > 0 gives
 *    AICDF_EINVAL.  Input and output byte ranges that overlap give
 *    AICDF_EALIAS (the paper's loops take restrict-qualified arrays, Code 1
 *    and Code 2).  Unsupported dtype combinations give AICDF_EDTYPE.
 *  - Values are not checked per element (hot path).  Inputs u are meant to be
 *    in (0,1); u = 0 and u = 1 give finite values of the capped table entries
 *    (or -inf/+inf for exact_icdf); NaN gives NaN for the dyadic and exact
 *    transforms and the first constant for the piecewise-constant one; other
 *    values outside [0,1] give finite, unspecified results.
 */
#ifndef AICDF_H
#define AICDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t aicdf_status;
#define AICDF_OK 0
#define AICDF_EINVAL (-1)   /* bad argument (NULL, size, range, enum)       */
#define AICDF_EDTYPE (-2)   /* unsupported dtype combination                */
#define AICDF_EALIAS (-3)   /* input and output memory overlap              */
#define AICDF_ENOMEM (-4)   /* host or device allocation failed             */
#define AICDF_EHIP (-5)     /* a HIP runtime call failed (see last_error)   */
#define AICDF_ERANGE (-6)   /* size beyond a documented maximum             */
#define AICDF_EIO (-7)      /* file could not be read or written            */

typedef enum {
  AICDF_F64 = 0,
  AICDF_F32 = 1,
  AICDF_F16 = 2,
  AICDF_BF16 = 3
} aicdf_dtype;

/* Thread-local description of the last failure in this thread ("" if none). */
const char* aicdf_last_error(void);

/* ------------------------------------------------------------------------ */
/* Coefficient tables                                                        */
/* ------------------------------------------------------------------------ */
typedef struct aicdf_table aicdf_table;

/* Piecewise-constant approximation on N = n_intervals equal intervals
 * [k/N, (k+1)/N) (Section 2.2, Theorem 2.3; Section 3.2).  construction:
 *   0  conditional mean E(Z | Phi(Z) in I_k)      (Corollary 2.4, "E"; the
 *      paper's choice)
 *   1  Phi^-1 of the interval midpoint            (Corollary 2.4, "C")
 *   2  Phi^-1 of the endpoint nearer 1/2          (Corollary 2.4, "I")
 * n_intervals: power of two in [2, 65536].  coef_t: F64, F32, F16 or BF16
 * (each constant is rounded to nearest even in coef_t).  The table is built
 * on the host in FP64 and copied to the current device.  *out receives the
 * handle.  Errors: EINVAL, EDTYPE, ENOMEM, EHIP. */
aicdf_status aicdf_table_const_create(uint32_t n_intervals, int32_t construction,
                                      aicdf_dtype coef_t, aicdf_table** out);

/* A piecewise-constant table with caller-given values on N equal intervals
 * (Section 2.2 includes moment-matching schemes as special cases; N = 2 with
 * values {-1, +1} gives the Rademacher variables of Section 1 and Table 3).
 * values: host array of N finite doubles, copied and rounded to coef_t.
 * n_intervals: power of two in [2, 65536].  Errors: EINVAL, EDTYPE, ENOMEM,
 * EHIP. */
aicdf_status aicdf_table_const_values(uint32_t n_intervals, const double* values, aicdf_dtype coef_t,
                                      aicdf_table** out);

/* Piecewise-polynomial approximation on dyadic intervals (Section 2.3,
 * Theorem 2.5 with decay rate r = 1/2; Section 3.3, Table 1).  A table of
 * T = n_entries rows serves u in (0, 1/2]:
 *   row 0        u = 1/2 exactly; all coefficients zero (Section 3.3)
 *   row e        [2^-(e+1), 2^-e) for 1 <= e <= T-2
 *   row T-1      the singular interval (0, 2^-(T-1))
 * u > 1/2 is served by antisymmetry.  Each row holds the L2-best polynomial
 * of the given degree on its interval, written in the local variable
 * s = u * 2^(e+1) (s in [1,2), or (0,2) on the singular row):
 *   D(u) = c_0 + c_1 s + ... + c_d s^d.
 * n_entries in [3, 64]; degree in [0, 3]; coef_t: F32, F16 or BF16.
 * Errors: EINVAL, EDTYPE, ENOMEM, EHIP. */
aicdf_status aicdf_table_dyadic_create(uint32_t n_entries, uint32_t degree,
                                       aicdf_dtype coef_t, aicdf_table** out);

/* Piecewise-polynomial approximation on geometric intervals with a general
 * decay rate r (Theorem 2.5).  With thresholds B_k = r^k / 2 (computed by
 * repeated FP64 multiplication from B_0 = 1/2 and rounded to FP32, so that a
 * FP32 input's row is decided by exact comparisons), T = n_entries rows serve
 * u in (0, 1/2]:
 *   row 0        u = 1/2 exactly; all coefficients zero
 *   row e        [B_e, B_(e-1)) for 1 <= e <= T-2
 *   row T-1      the singular interval (0, B_(T-2))
 * u > 1/2 is served by antisymmetry.  Each row holds the L2-best polynomial
 * of the given degree in s = u / B_e.  r = 1/2 reproduces the dyadic table
 * exactly.  The transform takes F32 input only: the row comes from a log2
 * estimate corrected against the thresholds, which costs more than the
 * dyadic exponent read (the trade-off of Section 3.3).
 * r in [0.05, 0.95]; n_entries in [3, 64] with r^(n_entries-1)/2 a normal
 * FP32 number; degree in [0, 3]; coef_t: F32, F16 or BF16.
 * Errors: EINVAL, EDTYPE, ENOMEM, EHIP. */
aicdf_status aicdf_table_geometric_create(double r, uint32_t n_entries, uint32_t degree, aicdf_dtype coef_t,
                                          aicdf_table** out);

/* The coef_t-rounded coefficients aicdf_table_geometric_create would store,
 * computed on the host, row-major T x (degree+1) into host_out
 * (cap >= T*(degree+1)); coef_t = F64 gives the unrounded FP64 fit.
 * Errors: EINVAL, EDTYPE, ERANGE. */
aicdf_status aicdf_table_geometric_host(double r, uint32_t n_entries, uint32_t degree, aicdf_dtype coef_t,
                                        double* host_out, size_t cap);

/* Copies the stored (coef_t-rounded) coefficients to host memory as doubles,
 * row-major rows x cols (constant tables: N x 1; dyadic and geometric:
 * T x (degree+1)).
 * host_out may be NULL to query rows/cols; otherwise cap >= rows*cols.
 * Errors: EINVAL, ERANGE. */
aicdf_status aicdf_table_coeffs(const aicdf_table* table, double* host_out, size_t cap,
                                uint32_t* rows, uint32_t* cols);

void aicdf_table_destroy(aicdf_table* table);

/* The same host FP64 construction without a device: writes the coef_t-rounded
 * coefficients that aicdf_table_const_create (kind 0; param = construction)
 * or aicdf_table_dyadic_create (kind 1; param = degree) would store, row-major,
 * to host_out (cap >= rows*cols: n for kind 0, n*(degree+1) for kind 1).
 * coef_t = F64 returns the unrounded FP64 fit for either kind.
 * Errors: EINVAL, EDTYPE, ERANGE. */
aicdf_status aicdf_table_host_coeffs(int32_t kind, uint32_t n, uint32_t param, aicdf_dtype coef_t,
                                     double* host_out, size_t cap);

/* ------------------------------------------------------------------------ */
/* Streaming transforms U -> Z (Section 3)                                   */
/* ------------------------------------------------------------------------ */

/* z[i] = Q[m] with m = min(floor(N u[i]), N-1) on a constant table (Code 1;
 * the clamp at N-1 covers u = 1, which the paper's loop leaves unguarded).
 * u: device, n elements of u_t; z: device, n elements of z_t.
 * (u_t, z_t) in {(F32,F32), (F32,F16), (F32,BF16), (F64,F32), (F64,F64)}.
 * Output rounding is to nearest even.  Asynchronous on `stream`.
 * Errors: EINVAL, EDTYPE, EALIAS, EHIP. */
aicdf_status approx_icdf_const(const aicdf_table* table, size_t n, const void* u, aicdf_dtype u_t,
                               void* z, aicdf_dtype z_t, void* stream);

/* Dyadic piecewise-polynomial transform (Algorithm 1): predicate u < 1/2,
 * reflection u' = 1 - u otherwise, row index e = min(B - 1 - E(u'), T - 1)
 * read from the biased exponent E of u' (B = 127 for F32 input, 1023 for
 * F64 input), s = u' 2^(e+1), Horner's rule with fused multiply-adds, sign
 * restored.  F32 input evaluates in FP32; F64 input evaluates in FP64 on the
 * stored coefficients.  Same dtype pairs, layout and errors as
 * approx_icdf_const.  On a geometric table (F32 input only, else EDTYPE) the
 * row is the e with B_e <= u' < B_(e-1) and s = u' (1/B_e) with the FP32
 * reciprocal of B_e. */
aicdf_status approx_icdf_linear(const aicdf_table* table, size_t n, const void* u, aicdf_dtype u_t,
                                void* z, aicdf_dtype z_t, void* stream);

/* The row (dyadic or geometric table) or interval (constant table) index
 * that the two transforms above select for each u, computed by the same
 * device code; for verifying the index step of Code 1 / Algorithm 1.
 * idx: device, n uint32.  u_t: F32 or F64 (F32 only for geometric tables).
 * Errors: EINVAL, EDTYPE, EALIAS, EHIP. */
aicdf_status approx_icdf_index(const aicdf_table* table, size_t n, const void* u, aicdf_dtype u_t,
                               uint32_t* idx, void* stream);

/* Exact inverse normal CDF Phi^-1 in FP64 (Section 3.1 describes the library
 * routines this stands for): Wichura's algorithm AS 241 (Applied Statistics
 * 37, 1988), rational functions of degree 7 in three regions of u, relative
 * error about 1e-16 (below 1e-15 measured against 50-digit roots).  The same
 * routine gives the exact normals of the fused GBM levels.
 * (u_t, z_t) in {(F64,F64), (F64,F32), (F32,F64), (F32,F32)}; u = 0 and
 * u = 1 give -inf and +inf.  Errors: EINVAL, EDTYPE, EALIAS, EHIP. */
aicdf_status exact_icdf(size_t n, const void* u, aicdf_dtype u_t, void* z, aicdf_dtype z_t,
                        void* stream);

/* Counter-based uniforms from Philox-4x32-10 (Salmon et al., SC'11).
 * Key (lo32(seed), hi32(seed)); counter words 2,3 = (lo32(stream_id),
 * hi32(stream_id)).
 *  F32: element i uses 32-bit word g = offset + i, from counter block g/4,
 *       word g mod 4; m = word >> 9; u = (m + 0.5) 2^-23 (odd multiples of
 *       2^-24, exact in FP32, never 0 or 1).
 *  F64: element i uses draw g = offset + i, counter block g/2, words
 *       2(g mod 2) (hi) and 2(g mod 2)+1 (lo); k = (hi:lo) >> 11;
 *       u = ((double)k + 0.5) 2^-53 rounded to nearest even, with the one
 *       value that rounds to 1.0 replaced by 1 - 2^-53.
 * u: device, n elements of u_t (F32 or F64).  Errors: EINVAL, EDTYPE, EHIP. */
aicdf_status aicdf_uniform_fill(uint64_t seed, uint64_t stream_id, uint64_t offset, size_t n,
                                void* u, aicdf_dtype u_t, void* stream);

/* Plain HBM streaming kernels that measure the achievable bandwidth which
 * bounds the transforms (the paper's "read and write" floor, Section 3.4).
 * mode 0: copy n_bytes from src to dst; mode 1: read n_bytes from src (dst
 * must hold 16 bytes and is written only in the impossible case that the
 * data fold to a sentinel); mode 2: write n_bytes to dst (src unused, may be
 * NULL).
 * n_bytes must be a multiple of 16 and both pointers 16-byte aligned.
 * Errors: EINVAL, EHIP. */
aicdf_status aicdf_bw_probe(int32_t mode, size_t n_bytes, const void* src, void* dst,
                            void* stream);

/* ------------------------------------------------------------------------ */
/* Nested multilevel Monte Carlo levels (Section 4, Section 5.2)             */
/* ------------------------------------------------------------------------ */
#define AICDF_KIND_EXACT 0      /* Y = P^_l - P^_(l-1), exact inverse        */
#define AICDF_KIND_APPROX 1     /* Y = P~_l - P~_(l-1), approximation        */
#define AICDF_KIND_CORRECTION 2 /* Y = P^_l - P^_(l-1) - P~_l + P~_(l-1)     */
#define AICDF_KIND_TWOWAY 3     /* CIR only: Y = P^_l - P~_l on the same draws,
                                   the two-way difference at one time step
                                   (Section 5.2, Figure 4b); P_f = P^_l and
                                   P_c = P~_l in the sums                     */

typedef struct {
  double S0, r, sigma, T, K; /* dX = r X dt + sigma X dW, X_0 = S0, strike K */
  int32_t scheme;            /* 0 Euler-Maruyama, 1 Milstein                 */
  int32_t payoff;            /* 0 P = X_T, 1 P = exp(-rT) max(X_T - K, 0)    */
} aicdf_gbm_params;

typedef struct {
  double v0, kappa, theta, xi, T; /* dv = kappa(theta - v)dt + xi sqrt(v) dW */
  int32_t functional;             /* 0 P = v_T, 1 trapezoidal time average  */
  int32_t reserved;               /* must be 0                              */
} aicdf_cir_params;

/* Compensated FP64 sums over the paths of one level call. */
typedef struct {
  double n;           /* number of paths                                     */
  double sum[4];      /* sum of Y, Y^2, Y^3, Y^4                             */
  double sum_pf;      /* sum of the fine functional (exact path for EXACT and
                         CORRECTION, approximate path for APPROX)            */
  double sum_pc;      /* sum of the coarse functional (0 at level 0)         */
  double kernel_ms;   /* device time of the level kernel, HIP events         */
  uint64_t fallbacks; /* CIR surrogate steps outside the trained log-lambda
                         range (lambda = 0 included), where the network is
                         evaluated at the range's nearer end                 */
  uint64_t reserved;
} aicdf_level_sums;

/* One MLMC level of geometric Brownian motion with the approximate normals
 * fused into the coupled fine/coarse paths (Section 4: Euler-Maruyama and
 * Milstein; the coarse Wiener increments are pairwise sums of the fine ones;
 * exact and approximate normals of one step come from one uniform).
 * level: 0..20 (2^level fine steps; no coarse path at level 0).
 * kind: AICDF_KIND_*.  approx: dyadic, geometric or constant table, required
 * unless kind == EXACT (ignored then); its normals are those of
 * approx_icdf_linear / approx_icdf_const on the same u24 values.
 * Paths path_offset .. path_offset+n_paths-1
 * of the stream (seed, level, kind) are simulated; any split of a path range
 * over calls gives the same per-path values, except that calls with
 * 2^level >= 4 and n_paths x G <= 2^19, G = min(64, 2^level / 2), run one
 * path per group of G lanes (each lane multiplies the linear step maps of
 * 2^level/G consecutive steps, and an ordered shuffle tree multiplies the
 * lane products), whose FP32 products round in another order: their per-path
 * values agree with the other launch shape to FP32 rounding.
 * Draws (Philox counter (block, lo32(path), hi32(path), level | kind << 8),
 * key seed): APPROX takes one 32-bit word per fine step (u24 grid as in
 * aicdf_uniform_fill F32); EXACT and CORRECTION take two words per step
 * (u53 grid as in aicdf_uniform_fill F64, and for CORRECTION the u24 of
 * the high word drives the approximate path).
 * out: host, receives the sums.  path_out: optional device buffer of
 * n_paths x 3 doubles (Y, P_f, P_c per path) or NULL.
 * Synchronises `stream`.  The library keeps one small workspace (~200 KB of
 * device memory) per (device, stream) that a level call has used, until the
 * process ends: level calls (GBM and CIR) on different streams, from
 * different host threads, run concurrently; calls on one stream are
 * serialised.  Errors: EINVAL, ERANGE, EHIP, ENOMEM. */
aicdf_status mlmc_level_gbm(const aicdf_gbm_params* params, uint32_t level, uint64_t n_paths,
                            int32_t kind, const aicdf_table* approx, uint64_t seed,
                            uint64_t path_offset, aicdf_level_sums* out, double* path_out,
                            void* stream);

typedef struct aicdf_surrogate aicdf_surrogate;

/* One MLMC level of the CIR process with exact-in-law non-central chi-squared
 * transitions (Section 5.2): with nu = 4 kappa theta / xi^2, per step of
 * delta = T / 2^level,  c = xi^2 (1 - e^(-kappa delta)) / (4 kappa),
 * lambda_n = v_n e^(-kappa delta) / c,  v_(n+1) = c C_nu^-1(U_n; lambda_n).
 * The coarse path is the fine path observed at even steps.  kind:
 *   EXACT       exact inverse (FP64), two-word u53 draws
 *   APPROX      the surrogate network (required), one-word u24 draws;
 *               outside the surrogate's log(lambda) range (lambda = 0
 *               included) the network is evaluated at the range's nearer
 *               end (below it P depends on lambda only through O(lambda)
 *               terms, above it P is close to its Gaussian limit); such
 *               steps are counted in out->fallbacks (the correction level
 *               removes the bias)
 *   CORRECTION  both on two-word draws (surrogate on the u24 of the high word)
 *   TWOWAY      both on the draws of CORRECTION, fine paths only:
 *               Y = P^_f - P~_f, sum_pf over P^_f, sum_pc over P~_f
 * Stream kinds are 4 + kind in the counter tag.  level 0..12.  Other
 * arguments as mlmc_level_gbm, with one qualification of split invariance:
 * EXACT, CORRECTION and TWOWAY calls with few paths run one path per
 * wavefront with a wave-cooperative exact inverse that sums in another
 * order: always at most 2048 paths, never 2^17 or more, and in between
 * below a cost model's crossover (it grows with lambda at the process level
 * max(v0, theta) and with the waves the kernel keeps resident); their
 * per-path values agree with those of the other shape to 1e-11 relative for
 * up to 16 steps, growing along longer paths (4e-11 measured at 256 steps):
 * each exact inverse's sums round differently, which can steer the root
 * iteration to another last step (the surrogate's values are
 * bit-identical).  Values are bit-identical between calls of the same
 * launch shape.  Errors: EINVAL, ERANGE, EHIP, ENOMEM. */
aicdf_status mlmc_level_cir(const aicdf_cir_params* params, uint32_t level, uint64_t n_paths,
                            int32_t kind, const aicdf_surrogate* approx, uint64_t seed,
                            uint64_t path_offset, aicdf_level_sums* out, double* path_out,
                            void* stream);

typedef struct aicdf_chi2_table aicdf_chi2_table;

/* As mlmc_level_cir with Section 5.1's piecewise-polynomial approximation in
 * place of the surrogate (the paper's own approximate CIR transition, Table 7
 * and Figure 4b): APPROX steps take x~ = max(C~^-1(u24; lambda), 0) in FP32
 * with no fallback (the knots cover every lambda >= 0); CORRECTION pairs it
 * with the exact FP64 inverse on the same draw.  `approx` must be built for
 * the process's nu = 4 kappa theta / xi^2 (relative difference <= 1e-12),
 * and is required unless kind == EXACT.  Draws and streams are those of
 * mlmc_level_cir.  Errors: EINVAL, ERANGE, EHIP, ENOMEM. */
aicdf_status mlmc_level_cir_table(const aicdf_cir_params* params, uint32_t level, uint64_t n_paths,
                                  int32_t kind, const aicdf_chi2_table* approx, uint64_t seed,
                                  uint64_t path_offset, aicdf_level_sums* out, double* path_out,
                                  void* stream);

/* As mlmc_level_cir with the truncated Euler-Maruyama scheme of Section 5.2
 * as the approximation (the Gaussian scheme of Figure 4b, not a chi-squared
 * approximation): APPROX steps take
 *   v' = v + kappa (theta - v) delta + xi sqrt(|v| delta) Phi^-1(u24)
 * with Phi^-1 in FP64 and v in FP32 (v may become negative; its modulus goes
 * under the root).  CORRECTION and TWOWAY pair it with the exact transition
 * on the same draw.  Errors: EINVAL, ERANGE, EHIP, ENOMEM. */
aicdf_status mlmc_level_cir_em(const aicdf_cir_params* params, uint32_t level, uint64_t n_paths,
                               int32_t kind, uint64_t seed, uint64_t path_offset,
                               aicdf_level_sums* out, double* path_out, void* stream);

/* As mlmc_level_cir with the Sankaran approximation (approx_ncx2_sankaran,
 * Section 5.1's comparator) as the approximate transition; CORRECTION and
 * TWOWAY pair it with the exact transition on the same draw.
 * Errors: EINVAL, ERANGE, EHIP, ENOMEM. */
aicdf_status mlmc_level_cir_sankaran(const aicdf_cir_params* params, uint32_t level, uint64_t n_paths,
                                     int32_t kind, uint64_t seed, uint64_t path_offset,
                                     aicdf_level_sums* out, double* path_out, void* stream);

/* Stream-ordered variants of the five level calls (Section 4.1's estimators
 * are sums over many independent level calls; these let one host thread
 * spread them over several streams).  Same arguments, checks, kernels and
 * per-path values as the synchronous call, except that the sums go to
 * sums_dev instead of a host struct: 8 doubles of device memory on the
 * current device, 8-byte aligned, owned by the caller, written by the device
 * in stream order as
 *   [0..3] sum Y, Y^2, Y^3, Y^4   [4] sum P_f   [5] sum P_c
 *   [6] fallbacks (exact integer)  [7] n_paths
 * bit-identical to the synchronous call's fields.  The call returns once the
 * work is enqueued: it neither waits for the device nor times the level
 * kernel.  sums_dev, path_out and the table or surrogate must stay valid
 * until `stream` has passed the call.  Calls on one stream use its workspace
 * one after another in stream order (no host wait between them); calls on
 * different streams run concurrently.  A zero-path call enqueues all-zero
 * sums.  Argument errors are returned before anything is enqueued.
 * Errors: EINVAL, ERANGE, EHIP, ENOMEM. */
aicdf_status mlmc_level_gbm_async(const aicdf_gbm_params* params, uint32_t level, uint64_t n_paths,
                                  int32_t kind, const aicdf_table* approx, uint64_t seed,
                                  uint64_t path_offset, double* sums_dev, double* path_out,
                                  void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mlmc_level_gbm_async with
 * the same arguments, checks, kernels and results (sums and per-path values
 * bit-identical), except that the level's per-work-group partial sums live in
 * a fixed array of device memory inside the library (192 KiB per GPU, at most
 * 4096 work-groups of 6 doubles, which every call's launch respects; a launch
 * needing more is rejected with ERANGE) instead of a per-stream workspace,
 * and that the fallback count (always 0 for GBM) is reported as 0.  The call
 * allocates nothing: no hipMalloc, hipFree, pinned or host allocation; on its
 * first call on a device it looks up that device's array (hipGetSymbolAddress).
 * Every call on one GPU shares that GPU's array, whatever the stream: calls
 * that overlap in time on one GPU (several streams, or host threads) race
 * and give wrong sums; serialise them, for example on one stream.  The final
 * pass reads only what the level kernel of the same call wrote.
 * Errors: EINVAL, ERANGE, EHIP. */
aicdf_status mlmc_level_gbm_noalloc(const aicdf_gbm_params* params, uint32_t level, uint64_t n_paths,
                                    int32_t kind, const aicdf_table* approx, uint64_t seed,
                                    uint64_t path_offset, double* sums_dev, double* path_out,
                                    void* stream);

/* One level job of a batched call: the arguments of one level call. */
typedef struct {
  uint32_t level;
  int32_t kind;         /* AICDF_KIND_EXACT, _APPROX or _CORRECTION */
  uint64_t n_paths;
  uint64_t path_offset;
} aicdf_level_job;

/* Several levels of one estimator in ONE launch (Section 4.1: an estimator is
 * a sum over levels and kinds, each level call a sum over its paths): the
 * level kernel runs every job, each on exactly the work-groups and paths its
 * own mlmc_level_gbm_async call would use, followed by one final pass with a
 * work-group per job, so every job's 8 sums are bit-identical to that call's
 * (per-path output is not offered).  Stream-ordered like
 * mlmc_level_gbm_async; sums_dev: device, n_jobs x 8 doubles in job order,
 * each row laid out as in that call.  jobs: host array of n_jobs <= 24
 * entries, read before the call returns; jobs of 0 paths give all-zero rows.
 * The jobs share params, approx and seed; kinds may be mixed (a nested
 * estimator's APPROX and CORRECTION levels in one launch).  Work-groups are
 * dispatched in job order, so put the longest jobs (the few-path high levels,
 * whose time is one path's serial time) first.  Uses the stream's workspace
 * (4.7 MB of batch partials, allocated on the first batched call).
 * Errors: EINVAL, ERANGE, EDTYPE, EHIP, ENOMEM (an error in job j names it). */
aicdf_status mlmc_levels_gbm(const aicdf_gbm_params* params, const aicdf_level_job* jobs, uint32_t n_jobs,
                             const aicdf_table* approx, uint64_t seed, double* sums_dev, void* stream);

/* The approximate transition of a batched CIR call (approx argument). */
#define AICDF_CIR_SURROGATE 0 /* const aicdf_surrogate*   (as mlmc_level_cir)          */
#define AICDF_CIR_TABLE 1     /* const aicdf_chi2_table*  (as mlmc_level_cir_table)    */
#define AICDF_CIR_EM 2        /* NULL                     (as mlmc_level_cir_em)       */
#define AICDF_CIR_SANKARAN 3  /* NULL                     (as mlmc_level_cir_sankaran) */

/* mlmc_levels_gbm for the CIR process (Section 5.2): every job of one
 * estimator in ONE launch of the level kernel plus one final pass; each job
 * runs on exactly the work-groups, launch shape and paths of its own
 * stream-ordered level call with the chosen approximation, so its 8 sums
 * (fallback count included) are bit-identical to that call's.  Kinds EXACT,
 * APPROX and CORRECTION (the two-way kind is not batched).  Arguments,
 * ordering advice, workspace and errors as for mlmc_levels_gbm; the
 * approximation is checked against params as in the level calls. */
aicdf_status mlmc_levels_cir(const aicdf_cir_params* params, const aicdf_level_job* jobs, uint32_t n_jobs,
                             int32_t approx_type, const void* approx, uint64_t seed, double* sums_dev,
                             void* stream);
aicdf_status mlmc_level_cir_async(const aicdf_cir_params* params, uint32_t level, uint64_t n_paths,
                                  int32_t kind, const aicdf_surrogate* approx, uint64_t seed,
                                  uint64_t path_offset, double* sums_dev, double* path_out,
                                  void* stream);
aicdf_status mlmc_level_cir_table_async(const aicdf_cir_params* params, uint32_t level,
                                        uint64_t n_paths, int32_t kind, const aicdf_chi2_table* table,
                                        uint64_t seed, uint64_t path_offset, double* sums_dev,
                                        double* path_out, void* stream);
aicdf_status mlmc_level_cir_em_async(const aicdf_cir_params* params, uint32_t level, uint64_t n_paths,
                                     int32_t kind, uint64_t seed, uint64_t path_offset,
                                     double* sums_dev, double* path_out, void* stream);
aicdf_status mlmc_level_cir_sankaran_async(const aicdf_cir_params* params, uint32_t level,
                                           uint64_t n_paths, int32_t kind, uint64_t seed,
                                           uint64_t path_offset, double* sums_dev, double* path_out,
                                           void* stream);

/* Optimal allocation of the nested estimator at RMSE eps (Section 4.1):
 *   T^ = 2 eps^-2 (sum_l sqrt(v^_l c^_l))^2,
 *   T~ = 2 eps^-2 (sum_l sqrt(v~_l c~_l) + sqrt(V~_l C~_l))^2,
 *   m^_l = eps^-1 sqrt(2 T^ v^_l / c^_l), m~_l = eps^-1 sqrt(2 T~ v~_l / c~_l),
 *   M~_l = eps^-1 sqrt(2 T~ V~_l / C~_l).
 * All arrays are host arrays of n_levels doubles; v_* >= 0, c_* > 0.  Any of
 * the m outputs may be NULL.  Errors: EINVAL. */
aicdf_status mlmc_allocate(uint32_t n_levels, double eps, const double* v_hat, const double* c_hat,
                           const double* v2, const double* c2, const double* v4, const double* c4,
                           double* m_hat, double* m2, double* m4, double* T_hat,
                           double* T_tilde);

/* ------------------------------------------------------------------------ */
/* Non-central chi-squared (Section 5)                                       */
/* ------------------------------------------------------------------------ */

/* x[i] = C_nu^-1(u[i]; lambda[i]) in FP64: the CDF is the Poisson mixture of
 * central chi-squared CDFs (Abramowitz & Stegun 26.4.25, which Section 5
 * cites), summed outward from the Poisson mode with incomplete-gamma
 * recurrences; the root is found by safeguarded third-order (Householder)
 * steps (with the density and its first two derivatives from the same
 * sweep) in log x on log C, or,
 * for 1 - u < 2^-10 (any u > 1/2 when lambda > 4096), in x on log(1 - C)
 * with 1 - C from the upward sweep,
 * inside a maintained bracket.
 * u, lambda, x: device arrays of n doubles; nu > 0; 0 <= lambda <= 1e8
 * (per element: a lambda outside that range, or NaN, gives x = NaN; the
 * series then needs more terms than the sweeps index).
 * u = 0 gives 0, u = 1 gives +inf.  Batches of n <= 8192 run one inverse per
 * wavefront (the sweeps split over the 64 lanes, for latency); larger ones
 * one per thread.  The two agree to 1e-11 relative (they round their sums
 * differently, which can change the last step of the root iteration).
 * Errors: EINVAL, EALIAS, EHIP. */
aicdf_status ncx2_icdf_exact(double nu, size_t n, const double* u, const double* lambda,
                             double* x, void* stream);

/* ------------------------------------------------------------------------ */
/* Piecewise-polynomial chi-squared approximation (Section 5.1)              */
/* ------------------------------------------------------------------------ */
/* At a fixed nu, C_nu^-1(U; lambda) = lambda + nu + 2 sqrt(lambda + nu) P(U; y)
 * with y = nu / (lambda + nu) in (0, 1].  The approximation P~ holds, at
 * n_knots knots equally spaced in sqrt(y) (sqrt(y_i) = i / (n_knots - 1);
 * y = 0 is the Gaussian limit Phi^-1, y = 1 the central chi-squared), two
 * dyadic piecewise polynomials of `degree` (1 or 3): one on U in (0, 1/2] in
 * t = U and one on U in (1/2, 1) in t = 1 - U, each with n_intervals
 * intervals [2^-(k+1), 2^-k), k = 1..n_intervals-1, and the singular
 * (0, 2^-n_intervals), fitted in L2 in s = t 2^(k+1).  Between knots P~ is
 * interpolated linearly in sqrt(y).  The paper's Table 6 uses 16 knots and
 * 15 intervals per half (the 16-entry layout of the normal tables).
 * Coefficient layout (FP64, host): [knot][half (0 lower, 1 upper)]
 * [interval k-1][degree+1], c_0 first.  The device copy is FP32.
 * Limits: nu in (0, 1e4], n_knots 2..64, n_intervals 2..30.  Building takes
 * 2 * n_knots * ~900 exact FP64 inversions on host threads (~0.1-1 s).
 * Errors: EINVAL, ENOMEM, EHIP. */
aicdf_status aicdf_chi2_table_create(double nu, uint32_t degree, uint32_t n_knots,
                                     uint32_t n_intervals, aicdf_chi2_table** out);
/* FP64 coefficients into host_out (cap doubles); *n_written (may be NULL)
 * receives the count; host_out == NULL only queries the count. */
aicdf_status aicdf_chi2_table_coeffs(const aicdf_chi2_table* t, double* host_out, size_t cap,
                                     size_t* n_written);
void aicdf_chi2_table_destroy(aicdf_chi2_table* t);
/* The same FP64 coefficients built on the host only (no device needed). */
aicdf_status aicdf_chi2_host_coeffs(double nu, uint32_t degree, uint32_t n_knots,
                                    uint32_t n_intervals, double* host_out, size_t cap);

/* x[i] = C~_nu^-1(u[i]; lambda[i]) in FP32 (u, lambda, x: device arrays of n
 * floats; x may not overlap an input).  lambda < 0 or NaN gives NaN; u
 * outside [0, 1] gives finite or NaN values without error; the formula
 * value is returned without clamping at 0.  Enqueues on `stream`.
 * Errors: EINVAL, EALIAS, EHIP. */
aicdf_status approx_ncx2_icdf(const aicdf_chi2_table* t, size_t n, const float* u,
                              const float* lambda, float* x, void* stream);

/* The Sankaran approximation, Section 5.1's comparator (Table 6d): with
 * k = nu, c1 = 1 - (2/3)(k+lambda)(k+3 lambda)/(k+2 lambda)^2,
 * c2 = (k+2 lambda)/(k+lambda)^2, c3 = (c1-1)(1-3 c1),
 *   x[i] = (k+lambda) max(B, 0)^(1/c1),
 *   B = 1 + c1 c2 (c1 - 1 + (2-c1) c2 c3/2) + c1 sqrt(2 c2)(1 + c2 c3/2) Phi^-1(u),
 * with Phi^-1 the exact FP64 inverse and the rest in FP32.  The Gaussian
 * term's root is sqrt(2 c2) and B is clamped at 0 (both as Table 6d fixes
 * them).  u, lambda, x: device arrays of n floats; nu in (0, 1e4].
 * lambda < 0 or NaN gives NaN.  Enqueues on `stream`.
 * Errors: EINVAL, EALIAS, EHIP. */
aicdf_status approx_ncx2_sankaran(double nu, size_t n, const float* u, const float* lambda, float* x,
                                  void* stream);

/* ------------------------------------------------------------------------ */
/* Learned surrogate for the CIR transition (MLP on BF16 MFMA)               */
/* ------------------------------------------------------------------------ */
/* The surrogate approximates Section 5.1's rescaled inverse
 *   P = (C_nu^-1(U; lambda) - lambda - nu) / (2 sqrt(lambda + nu))
 * at a fixed nu for log(lambda) in [loglam_lo, loglam_hi]:
 *   w  = D(U): the 16-row cubic dyadic approximation of Phi^-1 (FP32)
 *   g  = 2 (log lambda - loglam_lo) / (loglam_hi - loglam_lo) - 1
 *   h1 = relu(W1 [w, g] + b1)                 W1 64x2, FP32
 *   h2 = relu(W2 bf16(h1) + b2)               W2 64x64 in BF16, FP32 sums (MFMA)
 *   P~ = w + W3 . h2 + b3                     W3 64, FP32
 * relu(t) = max(t, 0).  Parameters are a flat FP32 vector of
 * AICDF_SURROGATE_NPARAMS values in the order W1 (row-major 64x2), b1, W2
 * (row-major 64x64, out x in), b2, W3, b3. */
#define AICDF_SURROGATE_HIDDEN 64
#define AICDF_SURROGATE_NPARAMS 4417

/* Creates a surrogate for degrees of freedom nu with a seeded uniform
 * +-1/sqrt(fan_in) initialisation.  Errors: EINVAL, ENOMEM, EHIP. */
aicdf_status aicdf_surrogate_create(double nu, double loglam_lo, double loglam_hi, uint64_t seed,
                                    aicdf_surrogate** out);
void aicdf_surrogate_destroy(aicdf_surrogate* s);

/* Host copies of the FP32 parameter vector (layout above); set also refreshes
 * the BF16 copy of W2 and resets the optimiser state.  Errors: EINVAL, EHIP. */
aicdf_status aicdf_surrogate_set_params(aicdf_surrogate* s, const float* host_params, size_t n);
aicdf_status aicdf_surrogate_get_params(const aicdf_surrogate* s, float* host_params, size_t n);

/* P~ for n inputs (device arrays of floats: u, log lambda -> p).  Inputs
 * outside the trained log-lambda range are evaluated anyway (no fallback).
 * Errors: EINVAL, EALIAS, EHIP. */
aicdf_status aicdf_surrogate_forward(const aicdf_surrogate* s, size_t n, const float* u,
                                     const float* loglam, float* p, void* stream);

/* Mean-squared-error loss against `target` (device) over n inputs and its
 * gradient with respect to every parameter (host, AICDF_SURROGATE_NPARAMS
 * floats), computed by the training kernels (BF16 layer-2 operands, FP32
 * sums, straight-through rounding).  Synchronises.  Errors: EINVAL, EHIP. */
aicdf_status aicdf_surrogate_loss_grad(const aicdf_surrogate* s, size_t n, const float* u,
                                       const float* loglam, const float* target,
                                       double* host_loss, float* host_grads, void* stream);

/* Training set: n samples with u on the u24 grid (a quarter of them pushed
 * into the tails by squaring, mirrored at random) and log lambda uniform on
 * the surrogate's range, from Philox stream (seed, 0x5EED); targets P from
 * the exact FP64 inverse.  Device arrays of n floats.  Errors: EINVAL, EHIP. */
aicdf_status aicdf_surrogate_make_data(const aicdf_surrogate* s, uint64_t seed, size_t n,
                                       float* u, float* loglam, float* target, void* stream);

/* Adam training (FP32 master weights) on device data for `epochs` passes of
 * mini-batches of `batch` samples (a multiple of 256, at most 262144) in a
 * seeded shuffled order; cosine learning-rate decay from lr.  host_loss
 * (optional) receives the mean loss of the last epoch.  Synchronises.
 * Errors: EINVAL, ENOMEM, EHIP. */
aicdf_status aicdf_surrogate_train(aicdf_surrogate* s, size_t n, const float* u,
                                   const float* loglam, const float* target, uint32_t epochs,
                                   uint32_t batch, float lr, uint64_t seed, double* host_loss,
                                   void* stream);

/* Range getters and persistence (little-endian header + FP32 parameters). */
aicdf_status aicdf_surrogate_info(const aicdf_surrogate* s, double* nu, double* loglam_lo,
                                  double* loglam_hi);
aicdf_status aicdf_surrogate_save(const aicdf_surrogate* s, const char* path);
aicdf_status aicdf_surrogate_load(const char* path, aicdf_surrogate** out);

#ifdef __cplusplus
}
#endif

#endif /* AICDF_H */
