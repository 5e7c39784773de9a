"""ctypes binding of libaicdf.so (argument marshalling only).

The shared library must have been built (python paper_2012_09715_amd/build.py);
there is no fallback path: loading fails loudly when it is missing.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaicdf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2012_09715_amd/build.py`")

lib = C.CDLL(LIB_PATH)

status = C.c_int32
vp = C.c_void_p
u32, u64, i32, sz, dbl, flt = C.c_uint32, C.c_uint64, C.c_int32, C.c_size_t, C.c_double, C.c_float
dptr = C.POINTER(C.c_double)
fptr = C.POINTER(C.c_float)


class GbmParams(C.Structure):
    _fields_ = [("S0", dbl), ("r", dbl), ("sigma", dbl), ("T", dbl), ("K", dbl),
                ("scheme", i32), ("payoff", i32)]


class CirParams(C.Structure):
    _fields_ = [("v0", dbl), ("kappa", dbl), ("theta", dbl), ("xi", dbl), ("T", dbl),
                ("functional", i32), ("reserved", i32)]


class LevelJob(C.Structure):
    _fields_ = [("level", u32), ("kind", i32), ("n_paths", u64), ("path_offset", u64)]


class LevelSums(C.Structure):
    _fields_ = [("n", dbl), ("sum", dbl * 4), ("sum_pf", dbl), ("sum_pc", dbl),
                ("kernel_ms", dbl), ("fallbacks", u64), ("reserved", u64)]


_PROTOS = {
    "aicdf_last_error": (C.c_char_p, []),
    "aicdf_table_const_create": (status, [u32, i32, i32, C.POINTER(vp)]),
    "aicdf_table_dyadic_create": (status, [u32, u32, i32, C.POINTER(vp)]),
    "aicdf_table_geometric_create": (status, [dbl, u32, u32, i32, C.POINTER(vp)]),
    "aicdf_table_geometric_host": (status, [dbl, u32, u32, i32, dptr, sz]),
    "aicdf_table_const_values": (status, [u32, dptr, i32, C.POINTER(vp)]),
    "aicdf_table_coeffs": (status, [vp, dptr, sz, C.POINTER(u32), C.POINTER(u32)]),
    "aicdf_table_destroy": (None, [vp]),
    "aicdf_table_host_coeffs": (status, [i32, u32, u32, i32, dptr, sz]),
    "approx_icdf_const": (status, [vp, sz, vp, i32, vp, i32, vp]),
    "approx_icdf_linear": (status, [vp, sz, vp, i32, vp, i32, vp]),
    "exact_icdf": (status, [sz, vp, i32, vp, i32, vp]),
    "approx_icdf_index": (status, [vp, sz, vp, i32, vp, vp]),
    "aicdf_uniform_fill": (status, [u64, u64, u64, sz, vp, i32, vp]),
    "aicdf_bw_probe": (status, [i32, sz, vp, vp, vp]),
    "mlmc_level_gbm": (status, [C.POINTER(GbmParams), u32, u64, i32, vp, u64, u64,
                                C.POINTER(LevelSums), vp, vp]),
    "mlmc_level_cir": (status, [C.POINTER(CirParams), u32, u64, i32, vp, u64, u64,
                                C.POINTER(LevelSums), vp, vp]),
    "mlmc_allocate": (status, [u32, dbl, dptr, dptr, dptr, dptr, dptr, dptr, dptr, dptr, dptr,
                               dptr, dptr]),
    "ncx2_icdf_exact": (status, [dbl, sz, vp, vp, vp, vp]),
    "aicdf_chi2_table_create": (status, [dbl, u32, u32, u32, C.POINTER(vp)]),
    "aicdf_chi2_table_coeffs": (status, [vp, dptr, sz, C.POINTER(sz)]),
    "aicdf_chi2_table_destroy": (None, [vp]),
    "aicdf_chi2_host_coeffs": (status, [dbl, u32, u32, u32, dptr, sz]),
    "approx_ncx2_icdf": (status, [vp, sz, vp, vp, vp, vp]),
    "mlmc_level_cir_table": (status, [C.POINTER(CirParams), u32, u64, i32, vp, u64, u64,
                                      C.POINTER(LevelSums), vp, vp]),
    "mlmc_level_cir_em": (status, [C.POINTER(CirParams), u32, u64, i32, u64, u64, C.POINTER(LevelSums), vp, vp]),
    "mlmc_level_cir_sankaran": (status, [C.POINTER(CirParams), u32, u64, i32, u64, u64, C.POINTER(LevelSums), vp,
                                         vp]),
    "mlmc_level_gbm_async": (status, [C.POINTER(GbmParams), u32, u64, i32, vp, u64, u64, vp, vp, vp]),
    "mlmc_levels_cir": (status, [C.POINTER(CirParams), C.POINTER(LevelJob), u32, i32, vp, u64, vp, vp]),
    "mlmc_levels_gbm": (status, [C.POINTER(GbmParams), C.POINTER(LevelJob), u32, vp, u64, vp, vp]),
    "mlmc_level_gbm_noalloc": (status, [C.POINTER(GbmParams), u32, u64, i32, vp, u64, u64, vp, vp, vp]),
    "mlmc_level_cir_async": (status, [C.POINTER(CirParams), u32, u64, i32, vp, u64, u64, vp, vp, vp]),
    "mlmc_level_cir_table_async": (status, [C.POINTER(CirParams), u32, u64, i32, vp, u64, u64, vp, vp, vp]),
    "mlmc_level_cir_em_async": (status, [C.POINTER(CirParams), u32, u64, i32, u64, u64, vp, vp, vp]),
    "mlmc_level_cir_sankaran_async": (status, [C.POINTER(CirParams), u32, u64, i32, u64, u64, vp, vp, vp]),
    "approx_ncx2_sankaran": (status, [dbl, sz, vp, vp, vp, vp]),
    "aicdf_surrogate_create": (status, [dbl, dbl, dbl, u64, C.POINTER(vp)]),
    "aicdf_surrogate_destroy": (None, [vp]),
    "aicdf_surrogate_set_params": (status, [vp, fptr, sz]),
    "aicdf_surrogate_get_params": (status, [vp, fptr, sz]),
    "aicdf_surrogate_forward": (status, [vp, sz, vp, vp, vp, vp]),
    "aicdf_surrogate_loss_grad": (status, [vp, sz, vp, vp, vp, dptr, fptr, vp]),
    "aicdf_surrogate_make_data": (status, [vp, u64, sz, vp, vp, vp, vp]),
    "aicdf_surrogate_train": (status, [vp, sz, vp, vp, vp, u32, u32, flt, u64, dptr, vp]),
    "aicdf_surrogate_info": (status, [vp, dptr, dptr, dptr]),
    "aicdf_surrogate_save": (status, [vp, C.c_char_p]),
    "aicdf_surrogate_load": (status, [C.c_char_p, C.POINTER(vp)]),
}

for _name, (_res, _args) in _PROTOS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EDTYPE", -3: "EALIAS", -4: "ENOMEM", -5: "EHIP",
                -6: "ERANGE", -7: "EIO"}


class AicdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != 0:
        raise AicdfError(code, lib.aicdf_last_error().decode())
