"""MI355X-native approximate inverse-CDF random variables and nested MLMC.

Python face of libaicdf.so (include/aicdf.h).  Every function marshals torch
tensors (device memory) and torch's current HIP stream into the C ABI; all
computation happens in the library's HIP kernels.  See the header for the
definitions, layouts and error behaviour of each call.
"""
import ctypes as C

import torch

from ._lib import (AicdfError, CirParams, GbmParams, LevelJob, LevelSums, check, lib)

F64, F32, F16, BF16 = 0, 1, 2, 3
KIND_EXACT, KIND_APPROX, KIND_CORRECTION, KIND_TWOWAY = 0, 1, 2, 3
SURROGATE_NPARAMS = 4417

_TORCH_TO_DT = {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
_DT_TO_TORCH = {v: k for k, v in _TORCH_TO_DT.items()}


def _dt(t):
    try:
        return _TORCH_TO_DT[t.dtype]
    except KeyError:
        raise AicdfError(-2, f"unsupported tensor dtype {t.dtype}") from None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, name, dtype=None, numel=None, like=None):
    """Device pointer of `t` after checking it: a contiguous CUDA tensor,
    of `dtype` if given, with at least `numel` elements if given, and on the
    device of `like` if given.  Raised before anything is launched, so that a
    wrong buffer never reaches a kernel."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise AicdfError(-1, f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise AicdfError(-1, f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise AicdfError(-2, f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise AicdfError(-1, f"{name} holds {t.numel()} elements, needs {numel}")
    if like is not None and t.device != like.device:
        raise AicdfError(-1, f"{name} is on {t.device}, expected {like.device}")
    return C.c_void_p(t.data_ptr())


def _path_out(path_out, n_paths):
    """Optional per-path output: float64, 3 doubles (Y, P_f, P_c) per path."""
    if path_out is None:
        return None
    return _dev(path_out, "path_out", torch.float64, 3 * int(n_paths))


class Table:
    """A coefficient table (library-owned; freed with the object)."""

    def __init__(self, handle, kind):
        self._h = handle
        self.kind = kind

    @property
    def handle(self):
        return self._h

    @classmethod
    def const(cls, n_intervals=1024, construction=0, coef_dtype=torch.float32):
        h = C.c_void_p()
        check(lib.aicdf_table_const_create(n_intervals, construction, _TORCH_TO_DT[coef_dtype], C.byref(h)))
        return cls(h, "const")

    @classmethod
    def const_values(cls, values, coef_dtype=torch.float32):
        """A piecewise-constant table with the given values (len a power of two)."""
        vals = [float(v) for v in values]
        h = C.c_void_p()
        check(lib.aicdf_table_const_values(len(vals), (C.c_double * len(vals))(*vals), _TORCH_TO_DT[coef_dtype],
                                           C.byref(h)))
        return cls(h, "const")

    @classmethod
    def rademacher(cls):
        """Rademacher variables (+-1 with probability 1/2): the 2-interval table {-1, +1}."""
        return cls.const_values([-1.0, 1.0])

    @classmethod
    def dyadic(cls, n_entries=16, degree=1, coef_dtype=torch.float32):
        h = C.c_void_p()
        check(lib.aicdf_table_dyadic_create(n_entries, degree, _TORCH_TO_DT[coef_dtype], C.byref(h)))
        return cls(h, "dyadic")

    @classmethod
    def geometric(cls, r=0.5, n_entries=16, degree=1, coef_dtype=torch.float32):
        """Piecewise polynomial on geometric intervals [r^e/2, r^(e-1)/2) (Theorem 2.5)."""
        h = C.c_void_p()
        check(lib.aicdf_table_geometric_create(float(r), n_entries, degree, _TORCH_TO_DT[coef_dtype], C.byref(h)))
        t = cls(h, "geometric")
        t.r = float(r)
        return t

    def coeffs(self):
        rows, cols = C.c_uint32(), C.c_uint32()
        check(lib.aicdf_table_coeffs(self._h, None, 0, C.byref(rows), C.byref(cols)))
        buf = (C.c_double * (rows.value * cols.value))()
        check(lib.aicdf_table_coeffs(self._h, buf, len(buf), None, None))
        return torch.tensor(list(buf), dtype=torch.float64).reshape(rows.value, cols.value)

    def __del__(self, _lib=lib):
        # _lib: bound at definition, since module globals may already be
        # cleared when objects are finalised at interpreter exit
        h, self._h = getattr(self, "_h", None), None
        if h:
            _lib.aicdf_table_destroy(h)


def table_host_coeffs(kind, n, param, coef_dtype=torch.float32):
    """Host-built coefficients (no device needed): kind "const" (param =
    construction) or "dyadic" (param = degree); rows x cols float64 tensor."""
    k = 0 if kind == "const" else 1
    cols = 1 if k == 0 else param + 1
    buf = (C.c_double * (n * cols))()
    check(lib.aicdf_table_host_coeffs(k, n, param, _TORCH_TO_DT[coef_dtype], buf, len(buf)))
    return torch.tensor(list(buf), dtype=torch.float64).reshape(n, cols)


def geometric_host_coeffs(r, n_entries, degree, coef_dtype=torch.float32):
    """Host-built coefficients of a geometric table (no device needed)."""
    buf = (C.c_double * (n_entries * (degree + 1)))()
    check(lib.aicdf_table_geometric_host(float(r), n_entries, degree, _TORCH_TO_DT[coef_dtype], buf, len(buf)))
    return torch.tensor(list(buf), dtype=torch.float64).reshape(n_entries, degree + 1)


def _out(u, z, out_dtype):
    if z is None:
        z = torch.empty(u.shape, dtype=out_dtype, device=u.device)
    else:
        _dev(z, "z", numel=u.numel(), like=u)
    return z


def approx_icdf_const(table, u, z=None, out_dtype=torch.float32, stream=None):
    z = _out(u, z, out_dtype)
    check(lib.approx_icdf_const(table.handle, u.numel(), _dev(u, "u"), _dt(u), _dev(z, "z"), _dt(z),
                                _stream(stream)))
    return z


def approx_icdf_linear(table, u, z=None, out_dtype=torch.float32, stream=None):
    z = _out(u, z, out_dtype)
    check(lib.approx_icdf_linear(table.handle, u.numel(), _dev(u, "u"), _dt(u), _dev(z, "z"), _dt(z),
                                 _stream(stream)))
    return z


def approx_icdf_index(table, u, stream=None):
    """Row/interval indices (int32 tensor holding the uint32 values)."""
    idx = torch.empty(u.shape, dtype=torch.int32, device=u.device)
    check(lib.approx_icdf_index(table.handle, u.numel(), _dev(u, "u"), _dt(u), _dev(idx, "idx"), _stream(stream)))
    return idx


def exact_icdf(u, z=None, out_dtype=torch.float64, stream=None):
    z = _out(u, z, out_dtype)
    check(lib.exact_icdf(u.numel(), _dev(u, "u"), _dt(u), _dev(z, "z"), _dt(z), _stream(stream)))
    return z


def uniform_fill(u, seed, stream_id=0, offset=0, stream=None):
    check(lib.aicdf_uniform_fill(seed, stream_id, offset, u.numel(), _dev(u, "u"), _dt(u), _stream(stream)))
    return u


def bw_probe(mode, src, dst, n_bytes=None, stream=None):
    nbytes = lambda t: t.numel() * t.element_size()
    nb = n_bytes if n_bytes is not None else (nbytes(dst) if mode != 1 else nbytes(src))
    if mode in (0, 1) and (src is None or nbytes(src) < nb):
        raise AicdfError(-1, f"src must hold {nb} bytes")
    if (mode != 1 and nbytes(dst) < nb) or nbytes(dst) < 16:
        raise AicdfError(-1, f"dst must hold {nb if mode != 1 else 16} bytes")
    s_ptr = _dev(src, "src") if src is not None else None
    check(lib.aicdf_bw_probe(mode, nb, s_ptr, _dev(dst, "dst"), _stream(stream)))


def _sums_dict(s):
    return {"n": s.n, "sum": list(s.sum), "sum_pf": s.sum_pf, "sum_pc": s.sum_pc,
            "kernel_ms": s.kernel_ms, "fallbacks": s.fallbacks}


def mlmc_level_gbm(params, level, n_paths, kind, table=None, seed=0, path_offset=0, path_out=None, stream=None):
    p = GbmParams(params["S0"], params["r"], params["sigma"], params["T"], params.get("K", 1.0),
                  int(params.get("scheme", 0)), int(params.get("payoff", 0)))
    out = LevelSums()
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_gbm(C.byref(p), level, n_paths, kind, table.handle if table is not None else None,
                             seed, path_offset, C.byref(out), po, _stream(stream)))
    return _sums_dict(out)


def mlmc_level_cir(params, level, n_paths, kind, surrogate=None, seed=0, path_offset=0, path_out=None,
                   stream=None):
    p = _cir_params(params)
    out = LevelSums()
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir(C.byref(p), level, n_paths, kind, surrogate.handle if surrogate is not None else None,
                             seed, path_offset, C.byref(out), po, _stream(stream)))
    return _sums_dict(out)


def _cir_params(params):
    return CirParams(params["v0"], params["kappa"], params["theta"], params["xi"], params["T"],
                     int(params.get("functional", 0)), 0)


def mlmc_level_cir_table(params, level, n_paths, kind, table=None, seed=0, path_offset=0, path_out=None,
                         stream=None):
    """mlmc_level_cir with the piecewise-polynomial chi-squared table (Chi2Table) as the approximation."""
    p = _cir_params(params)
    out = LevelSums()
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_table(C.byref(p), level, n_paths, kind, table.handle if table is not None else None,
                                   seed, path_offset, C.byref(out), po, _stream(stream)))
    return _sums_dict(out)


def mlmc_level_cir_em(params, level, n_paths, kind, seed=0, path_offset=0, path_out=None, stream=None):
    """mlmc_level_cir with the truncated Euler-Maruyama scheme as the approximation."""
    p = _cir_params(params)
    out = LevelSums()
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_em(C.byref(p), level, n_paths, kind, seed, path_offset, C.byref(out), po,
                                _stream(stream)))
    return _sums_dict(out)


def mlmc_level_cir_sankaran(params, level, n_paths, kind, seed=0, path_offset=0, path_out=None, stream=None):
    """mlmc_level_cir with the Sankaran approximation as the approximate transition."""
    p = _cir_params(params)
    out = LevelSums()
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_sankaran(C.byref(p), level, n_paths, kind, seed, path_offset, C.byref(out), po,
                                      _stream(stream)))
    return _sums_dict(out)


def _sums_dev(sums):
    if not isinstance(sums, torch.Tensor) or sums.dtype != torch.float64 or sums.numel() < 8:
        raise AicdfError(-1, "sums must be a float64 CUDA tensor of at least 8 elements")
    return _dev(sums, "sums")


def sums_dict(row):
    """The 8 doubles a stream-ordered level call writes (host array or tensor),
    as the synchronous calls' result dict (no device time: kernel_ms None)."""
    r = [float(v) for v in (row.tolist() if hasattr(row, "tolist") else row)]
    return {"n": r[7], "sum": r[0:4], "sum_pf": r[4], "sum_pc": r[5], "kernel_ms": None, "fallbacks": int(r[6])}


def mlmc_level_gbm_async(params, level, n_paths, kind, table, seed, path_offset, sums, path_out=None, stream=None):
    """Stream-ordered mlmc_level_gbm: enqueues the level on `stream` (default:
    the current stream) and returns; the device writes the 8 sums into `sums`
    (a float64 CUDA tensor).  `table`, `sums` and `path_out` must stay alive
    until the stream has passed the call."""
    p = GbmParams(params["S0"], params["r"], params["sigma"], params["T"], params.get("K", 1.0),
                  int(params.get("scheme", 0)), int(params.get("payoff", 0)))
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_gbm_async(C.byref(p), level, n_paths, kind, table.handle if table is not None else None,
                                   seed, path_offset, _sums_dev(sums), po, _stream(stream)))


MAX_JOBS = 24


def _jobs(jobs):
    """(level, kind, n_paths, path_offset) tuples -> a ctypes LevelJob array."""
    jobs = list(jobs)
    arr = (LevelJob * max(len(jobs), 1))()
    for i, (level, kind, n, off) in enumerate(jobs):
        arr[i] = LevelJob(int(level), int(kind), int(n), int(off))
    return arr, len(jobs)


def _batch_sums(sums, n_jobs):
    if not isinstance(sums, torch.Tensor) or sums.dtype != torch.float64 or sums.numel() < 8 * n_jobs:
        raise AicdfError(-1, f"sums must be a float64 CUDA tensor of at least {8 * n_jobs} elements")
    return _dev(sums, "sums")


def mlmc_levels_gbm(params, jobs, table, seed, sums, stream=None):
    """Several GBM levels in one launch (stream-ordered): jobs is a list of
    (level, kind, n_paths, path_offset); row j of `sums` (n_jobs x 8 float64
    on the device) receives job j's 8 sums, bit-identical to its
    mlmc_level_gbm_async call."""
    p = GbmParams(params["S0"], params["r"], params["sigma"], params["T"], params.get("K", 1.0),
                  int(params.get("scheme", 0)), int(params.get("payoff", 0)))
    arr, n = _jobs(jobs)
    check(lib.mlmc_levels_gbm(C.byref(p), arr, n, table.handle if table is not None else None, seed,
                              _batch_sums(sums, n), _stream(stream)))


CIR_SURROGATE, CIR_TABLE, CIR_EM, CIR_SANKARAN = 0, 1, 2, 3


def mlmc_levels_cir(params, jobs, approx, seed, sums, stream=None):
    """Several CIR levels in one launch (stream-ordered): jobs as for
    mlmc_levels_gbm; approx is a Surrogate, a Chi2Table, "em", "sankaran" or
    None (EXACT jobs only)."""
    p = _cir_params(params)
    arr, n = _jobs(jobs)
    if isinstance(approx, Surrogate):
        t, h = CIR_SURROGATE, approx.handle
    elif isinstance(approx, Chi2Table):
        t, h = CIR_TABLE, approx.handle
    elif approx == "em":
        t, h = CIR_EM, None
    elif approx == "sankaran":
        t, h = CIR_SANKARAN, None
    elif approx is None:
        t, h = CIR_SURROGATE, None
    else:
        raise AicdfError(-1, f"unknown approximation {approx!r}")
    check(lib.mlmc_levels_cir(C.byref(p), arr, n, t, h, seed, _batch_sums(sums, n), _stream(stream)))


def mlmc_level_gbm_noalloc(params, level, n_paths, kind, table, seed, path_offset, sums, path_out=None,
                           stream=None):
    """mlmc_level_gbm_async without any allocation: the level's partial sums
    live in the library's fixed per-GPU scratch array, shared by every call on
    that GPU (calls that overlap in time on one GPU race)."""
    p = GbmParams(params["S0"], params["r"], params["sigma"], params["T"], params.get("K", 1.0),
                  int(params.get("scheme", 0)), int(params.get("payoff", 0)))
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_gbm_noalloc(C.byref(p), level, n_paths, kind, table.handle if table is not None else None,
                                     seed, path_offset, _sums_dev(sums), po, _stream(stream)))


def mlmc_level_cir_async(params, level, n_paths, kind, surrogate, seed, path_offset, sums, path_out=None,
                         stream=None):
    """Stream-ordered mlmc_level_cir (see mlmc_level_gbm_async)."""
    p = _cir_params(params)
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_async(C.byref(p), level, n_paths, kind,
                                   surrogate.handle if surrogate is not None else None, seed, path_offset,
                                   _sums_dev(sums), po, _stream(stream)))


def mlmc_level_cir_table_async(params, level, n_paths, kind, table, seed, path_offset, sums, path_out=None,
                               stream=None):
    """Stream-ordered mlmc_level_cir_table (see mlmc_level_gbm_async)."""
    p = _cir_params(params)
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_table_async(C.byref(p), level, n_paths, kind, table.handle if table is not None else None,
                                         seed, path_offset, _sums_dev(sums), po, _stream(stream)))


def mlmc_level_cir_em_async(params, level, n_paths, kind, seed, path_offset, sums, path_out=None, stream=None):
    """Stream-ordered mlmc_level_cir_em (see mlmc_level_gbm_async)."""
    p = _cir_params(params)
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_em_async(C.byref(p), level, n_paths, kind, seed, path_offset, _sums_dev(sums), po,
                                      _stream(stream)))


def mlmc_level_cir_sankaran_async(params, level, n_paths, kind, seed, path_offset, sums, path_out=None,
                                  stream=None):
    """Stream-ordered mlmc_level_cir_sankaran (see mlmc_level_gbm_async)."""
    p = _cir_params(params)
    po = _path_out(path_out, n_paths)
    check(lib.mlmc_level_cir_sankaran_async(C.byref(p), level, n_paths, kind, seed, path_offset, _sums_dev(sums),
                                            po, _stream(stream)))


def approx_ncx2_sankaran(nu, u, lam, x=None, stream=None):
    """The Sankaran approximation x~(u; lambda) in FP32 (u, lambda: float32 device tensors)."""
    if u.dtype != torch.float32 or lam.dtype != torch.float32:
        raise AicdfError(-2, "u and lambda must be float32")
    if u.numel() != lam.numel():
        raise AicdfError(-1, "u and lambda must have the same number of elements")
    if x is None:
        x = torch.empty_like(u)
    elif x.dtype != torch.float32 or x.numel() != u.numel():
        raise AicdfError(-2, "x must be float32 with as many elements as u")
    check(lib.approx_ncx2_sankaran(nu, u.numel(), _dev(u, "u"), _dev(lam, "lambda", like=u), _dev(x, "x", like=u),
                                   _stream(stream)))
    return x


def mlmc_allocate(eps, v_hat, c_hat, v2, c2, v4, c4):
    n = len(v_hat)
    arr = lambda xs: (C.c_double * n)(*[float(x) for x in xs])
    mh, m2, m4 = (C.c_double * n)(), (C.c_double * n)(), (C.c_double * n)()
    Th, Tt = C.c_double(), C.c_double()
    check(lib.mlmc_allocate(n, eps, arr(v_hat), arr(c_hat), arr(v2), arr(c2), arr(v4), arr(c4), mh, m2, m4,
                            C.byref(Th), C.byref(Tt)))
    return {"m_hat": list(mh), "m_tilde": list(m2), "M_tilde": list(m4), "T_hat": Th.value, "T_tilde": Tt.value}


def ncx2_icdf_exact(nu, u, lam, x=None, stream=None):
    """x = C_nu^-1(u; lambda) in FP64 (u, lambda, x: float64 device tensors of one size)."""
    n = u.numel()
    pu = _dev(u, "u", torch.float64)
    if lam.numel() != n:
        raise AicdfError(-1, "u and lambda must have the same number of elements")
    pl = _dev(lam, "lambda", torch.float64, like=u)
    if x is None:
        x = torch.empty_like(u)
    px = _dev(x, "x", torch.float64, n, like=u)
    check(lib.ncx2_icdf_exact(nu, n, pu, pl, px, _stream(stream)))
    return x


class Chi2Table:
    """Piecewise-polynomial approximation of the non-central chi-squared
    inverse CDF at a fixed nu (library-owned handle)."""

    def __init__(self, handle, nu, degree, n_knots, n_intervals):
        self._h = handle
        self.nu, self.degree, self.n_knots, self.n_intervals = nu, degree, n_knots, n_intervals

    @property
    def handle(self):
        return self._h

    @classmethod
    def create(cls, nu, degree=1, n_knots=16, n_intervals=15):
        h = C.c_void_p()
        check(lib.aicdf_chi2_table_create(nu, degree, n_knots, n_intervals, C.byref(h)))
        return cls(h, nu, degree, n_knots, n_intervals)

    def coeffs(self):
        """FP64 coefficients, shape (n_knots, 2, n_intervals, degree + 1)."""
        n = C.c_size_t()
        check(lib.aicdf_chi2_table_coeffs(self._h, None, 0, C.byref(n)))
        buf = (C.c_double * n.value)()
        check(lib.aicdf_chi2_table_coeffs(self._h, buf, n.value, None))
        return torch.tensor(list(buf), dtype=torch.float64).reshape(self.n_knots, 2, self.n_intervals,
                                                                    self.degree + 1)

    def __del__(self, _lib=lib):
        # _lib: bound at definition, since module globals may already be
        # cleared when objects are finalised at interpreter exit
        h, self._h = getattr(self, "_h", None), None
        if h:
            _lib.aicdf_chi2_table_destroy(h)


def chi2_host_coeffs(nu, degree=1, n_knots=16, n_intervals=15):
    """The FP64 coefficients built on the host only (no device)."""
    n = n_knots * 2 * n_intervals * (degree + 1)
    buf = (C.c_double * n)()
    check(lib.aicdf_chi2_host_coeffs(nu, degree, n_knots, n_intervals, buf, n))
    return torch.tensor(list(buf), dtype=torch.float64).reshape(n_knots, 2, n_intervals, degree + 1)


def approx_ncx2_icdf(table, u, lam, x=None, stream=None):
    """x~ = C~^-1(u; lambda) in FP32 (u, lambda: float32 device tensors)."""
    if u.dtype != torch.float32 or lam.dtype != torch.float32:
        raise AicdfError(-2, "u and lambda must be float32")
    if u.numel() != lam.numel():
        raise AicdfError(-1, "u and lambda must have the same number of elements")
    if x is None:
        x = torch.empty_like(u)
    elif x.dtype != torch.float32 or x.numel() != u.numel():
        raise AicdfError(-2, "x must be float32 with as many elements as u")
    check(lib.approx_ncx2_icdf(table.handle, u.numel(), _dev(u, "u"), _dev(lam, "lambda", like=u),
                               _dev(x, "x", like=u), _stream(stream)))
    return x


class Surrogate:
    """The MLP surrogate of the CIR transition (library-owned handle)."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    @classmethod
    def create(cls, nu, loglam_lo, loglam_hi, seed=0):
        h = C.c_void_p()
        check(lib.aicdf_surrogate_create(nu, loglam_lo, loglam_hi, seed, C.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        check(lib.aicdf_surrogate_load(str(path).encode(), C.byref(h)))
        return cls(h)

    def save(self, path):
        check(lib.aicdf_surrogate_save(self._h, str(path).encode()))

    def info(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        check(lib.aicdf_surrogate_info(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def get_params(self):
        buf = (C.c_float * SURROGATE_NPARAMS)()
        check(lib.aicdf_surrogate_get_params(self._h, buf, SURROGATE_NPARAMS))
        return torch.tensor(list(buf), dtype=torch.float32)

    def set_params(self, flat):
        flat = [float(x) for x in flat]
        buf = (C.c_float * len(flat))(*flat)
        check(lib.aicdf_surrogate_set_params(self._h, buf, len(flat)))

    @staticmethod
    def _f32(u, **others):
        """Pointers of float32 device tensors of u's size (u first)."""
        n = u.numel()
        ptrs = [_dev(u, "u", torch.float32)]
        for name, t in others.items():
            if t.numel() != n:
                raise AicdfError(-1, f"{name} must have as many elements as u")
            ptrs.append(_dev(t, name, torch.float32, like=u))
        return ptrs

    def forward(self, u, loglam, p=None, stream=None):
        if p is None:
            p = torch.empty_like(u)
        pu, pg, pp = self._f32(u, loglam=loglam, p=p)
        check(lib.aicdf_surrogate_forward(self._h, u.numel(), pu, pg, pp, _stream(stream)))
        return p

    def loss_grad(self, u, loglam, target, stream=None):
        loss = C.c_double()
        g = (C.c_float * SURROGATE_NPARAMS)()
        pu, pg, pt = self._f32(u, loglam=loglam, target=target)
        check(lib.aicdf_surrogate_loss_grad(self._h, u.numel(), pu, pg, pt, C.byref(loss), g, _stream(stream)))
        return loss.value, torch.tensor(list(g), dtype=torch.float32)

    def make_data(self, n, seed, device="cuda", stream=None):
        u = torch.empty(n, dtype=torch.float32, device=device)
        g = torch.empty_like(u)
        t = torch.empty_like(u)
        check(lib.aicdf_surrogate_make_data(self._h, seed, n, _dev(u, "u"), _dev(g, "loglam"), _dev(t, "target"),
                                            _stream(stream)))
        return u, g, t

    def train(self, u, loglam, target, epochs, batch=4096, lr=1e-3, seed=0, stream=None):
        loss = C.c_double()
        pu, pg, pt = self._f32(u, loglam=loglam, target=target)
        check(lib.aicdf_surrogate_train(self._h, u.numel(), pu, pg, pt, epochs, batch, lr, seed, C.byref(loss),
                                        _stream(stream)))
        return loss.value

    def __del__(self, _lib=lib):
        # _lib: bound at definition, since module globals may already be
        # cleared when objects are finalised at interpreter exit
        h, self._h = getattr(self, "_h", None), None
        if h:
            _lib.aicdf_surrogate_destroy(h)
