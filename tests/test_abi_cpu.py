"""The C ABI on the CPU: every declared symbol is exported, host-side logic
(table construction, allocation, argument checks) works without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import torch

import paper_2012_09715_amd as A
from paper_2012_09715_amd._lib import lib
from oracle import mlmc, tables
from oracle.dtypes import ROUND

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "aicdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:aicdf_status|void|const char\s*\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("T", [8, 16, 32])
@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_host_dyadic_fit_matches_oracle(T, d):
    lib64 = A.table_host_coeffs("dyadic", T, d, torch.float64).numpy()
    ref = tables.dyadic_table(T, d)
    # the cubic normal equations amplify quadrature error: both fits sit ~2e-10
    # from a 40-digit mpmath fit at T = 32, far below FP32 resolution
    assert np.allclose(lib64, ref, rtol=1e-9, atol=1e-9)
    for dt, name in ((torch.float32, "f32"), (torch.float16, "f16"), (torch.bfloat16, "bf16")):
        got = A.table_host_coeffs("dyadic", T, d, dt).numpy()
        want = ROUND[name](ref)
        # identical rounding unless the FP64 fits straddle a rounding boundary
        mism = got != want
        assert mism.sum() <= 1
        if mism.any():
            assert np.all(np.abs(got - want)[mism] <= np.spacing(np.abs(want[mism]).astype(np.float32)) * (1 << 16))


@pytest.mark.parametrize("N", [2, 16, 1024, 65536])
@pytest.mark.parametrize("construction", [0, 1, 2])
def test_host_const_table_matches_oracle(N, construction):
    got = A.table_host_coeffs("const", N, construction, torch.float64).numpy().ravel()
    ref = tables.const_table(N, "ECI"[construction])
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-11)
    assert np.array_equal(got, -got[::-1])


def test_host_coeffs_argument_errors():
    buf = (C.c_double * 16)()
    assert lib.aicdf_table_host_coeffs(0, 1000, 0, 1, buf, 16) == -1  # not a power of two
    assert lib.aicdf_table_host_coeffs(1, 16, 4, 1, buf, 64) == -1    # degree 4
    assert lib.aicdf_table_host_coeffs(1, 16, 1, 1, buf, 16) == -6    # cap too small
    assert "cap" in lib.aicdf_last_error().decode()
    assert lib.aicdf_table_host_coeffs(1, 16, 1, 9, buf, 64) == -2    # bad dtype


def test_table_create_argument_errors_need_no_device():
    h = C.c_void_p()
    assert lib.aicdf_table_const_create(3, 0, 1, C.byref(h)) == -1
    assert lib.aicdf_table_dyadic_create(16, 1, 0, C.byref(h)) == -2
    assert lib.aicdf_table_dyadic_create(2, 1, 1, C.byref(h)) == -1
    assert not h.value
    lib.aicdf_table_destroy(None)  # no-op


def test_transform_argument_errors_need_no_device():
    assert lib.approx_icdf_linear(None, 10, None, 1, None, 1, None) == -1
    assert lib.exact_icdf(0, None, 1, None, 1, None) == 0          # n = 0 no-op
    assert lib.exact_icdf(10, None, 1, None, 1, None) == -1        # NULL with n > 0
    assert lib.exact_icdf(10, C.c_void_p(4096), 7, C.c_void_p(8192), 1, None) == -2
    # overlapping ranges
    assert lib.exact_icdf(100, C.c_void_p(4096), 0, C.c_void_p(4096 + 8), 0, None) == -3
    assert lib.aicdf_uniform_fill(1, 0, 0, 10, C.c_void_p(4096), 2, None) == -2
    assert lib.aicdf_bw_probe(0, 17, C.c_void_p(4096), C.c_void_p(8192), None) == -1


def test_async_level_argument_errors_need_no_device():
    from paper_2012_09715_amd._lib import CirParams, GbmParams
    g = GbmParams(1.0, 0.05, 0.2, 1.0, 1.0, 0, 1)
    c = CirParams(0.04, 0.5, 0.04, 0.3, 1.0, 1, 0)
    # NULL or misaligned sums_dev, before any device call
    assert lib.mlmc_level_gbm_async(C.byref(g), 2, 100, 0, None, 1, 0, None, None, None) == -1
    assert lib.mlmc_level_gbm_async(C.byref(g), 2, 100, 0, None, 1, 0, C.c_void_p(4100), None, None) == -1
    assert b"aligned" in lib.aicdf_last_error()
    assert lib.mlmc_level_cir_async(C.byref(c), 2, 100, 0, None, 1, 0, None, None, None) == -1
    assert lib.mlmc_level_cir_table_async(C.byref(c), 2, 100, 0, None, 1, 0, C.c_void_p(4097), None, None) == -1
    assert lib.mlmc_level_cir_em_async(C.byref(c), 2, 100, 0, 1, 0, None, None, None) == -1
    assert lib.mlmc_level_cir_sankaran_async(None, 2, 100, 0, 1, 0, C.c_void_p(4096), None, None) == -1
    # the synchronous calls still require their host output
    assert lib.mlmc_level_gbm(C.byref(g), 2, 100, 0, None, 1, 0, None, None, None) == -1


def test_mlmc_allocate_matches_oracle():
    rng = np.random.default_rng(3)
    for _ in range(10):
        L = int(rng.integers(1, 12))
        vh, ch = rng.random(L), rng.random(L) + 0.1
        v2, c2 = vh * 1.01, ch / 7
        v4, c4 = vh * 2.0 ** -14, ch + c2
        got = A.mlmc_allocate(1e-3, vh, ch, v2, c2, v4, c4)
        ref = mlmc.allocation(1e-3, vh, ch, v2, c2, v4, c4)
        assert got["T_hat"] == pytest.approx(ref["T_hat"], rel=1e-12)
        assert got["T_tilde"] == pytest.approx(ref["T_tilde"], rel=1e-12)
        for k in ("m_hat", "m_tilde", "M_tilde"):
            assert np.allclose(got[k], ref[k], rtol=1e-12)


def test_mlmc_allocate_table3_row():
    # the paper's Table 3 linear row from the library's allocation
    r = A.mlmc_allocate(1.0, [1.0], [7.0], [1.0], [1.0], [2.0 ** -14], [8.0])
    assert round(r["T_hat"] / r["T_tilde"], 2) == 6.70
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_allocate(1e-3, [1.0], [0.0], [1.0], [1.0], [1.0], [1.0])


@pytest.mark.parametrize("nu,degree", [(1.0, 1), (0.8888888888888888, 1), (5.0, 3), (100.0, 3), (0.3, 3)])
def test_host_chi2_table_matches_oracle(nu, degree):
    # The library's chi-squared tables (its own quadrature and exact inverse)
    # against the oracle's (Section 5.1): the cubic normal equations amplify
    # quadrature differences to ~1e-9, far below FP32 resolution.
    from oracle import chi2table
    got = A.chi2_host_coeffs(nu, degree).numpy()
    ref = chi2table.build(nu, degree)
    assert got.shape == ref.shape == (16, 2, 15, degree + 1)
    tol = 1e-11 if degree == 1 else 5e-9
    assert np.allclose(got, ref, rtol=0, atol=tol)


def test_host_chi2_table_shapes_and_errors():
    from oracle import chi2table
    got = A.chi2_host_coeffs(2.0, 1, n_knots=5, n_intervals=7).numpy()
    ref = chi2table.build(2.0, 1, n_knots=5, n_int=7)
    assert np.allclose(got, ref, rtol=0, atol=1e-11)
    buf = (C.c_double * 4)()
    for args in ((0.0, 1, 16, 15), (1.0, 2, 16, 15), (1.0, 1, 1, 15), (1.0, 1, 65, 15), (1.0, 1, 16, 1),
                 (1.0, 1, 16, 31), (float("nan"), 1, 16, 15)):
        assert lib.aicdf_chi2_host_coeffs(*args, buf, 4) == -1, args
    assert lib.aicdf_chi2_host_coeffs(1.0, 1, 2, 2, buf, 4) == -1  # needs 16 doubles
    assert lib.aicdf_chi2_host_coeffs(1.0, 1, 2, 2, None, 16) == -1


def test_const_values_argument_errors():
    h = C.c_void_p()
    vals = (C.c_double * 4)(-1.0, 0.0, 1.0, 2.0)
    assert lib.aicdf_table_const_values(3, vals, 1, C.byref(h)) == -1  # not a power of two
    assert lib.aicdf_table_const_values(4, None, 1, C.byref(h)) == -1
    assert lib.aicdf_table_const_values(4, vals, 9, C.byref(h)) == -2
    bad = (C.c_double * 2)(1.0, float("nan"))
    assert lib.aicdf_table_const_values(2, bad, 1, C.byref(h)) == -1


@pytest.mark.parametrize("r,T", [(0.5, 16), (0.3, 40), (0.7, 64), (0.95, 64)])
@pytest.mark.parametrize("d", [0, 1, 3])
def test_host_geometric_fit_matches_oracle(r, T, d):
    # compared as functions on each row: for r near 1 the monomial basis in
    # s on [1, 1/r) is ill-conditioned, so two accurate fits can differ in
    # their coefficients while agreeing as polynomials
    lib64 = A.geometric_host_coeffs(r, T, d, torch.float64).numpy()
    ref = tables.geometric_table(r, T, d)
    for e in range(1, T):
        a, b, h = tables.geometric_interval(e, r, T)
        s = np.linspace(a / h, b / h, 17)
        assert np.allclose(np.polyval(lib64[e][::-1], s), np.polyval(ref[e][::-1], s), rtol=0, atol=1e-10), e
    if r == 0.5:
        # the dyadic builder solves the monomial normal equations (~1e-10 for cubics)
        assert np.allclose(lib64, A.table_host_coeffs("dyadic", T, d, torch.float64).numpy(), rtol=1e-9, atol=1e-9)
    for dt, name in ((torch.float32, "f32"), (torch.bfloat16, "bf16")):
        assert np.array_equal(A.geometric_host_coeffs(r, T, d, dt).numpy(), ROUND[name](lib64))


def test_host_geometric_argument_errors():
    buf = (C.c_double * 256)()
    f = lib.aicdf_table_geometric_host
    assert f(0.04, 16, 1, 1, buf, 256) == -1      # r below 0.05
    assert f(0.96, 16, 1, 1, buf, 256) == -1      # r above 0.95
    assert f(float("nan"), 16, 1, 1, buf, 256) == -1
    assert f(0.7, 2, 1, 1, buf, 256) == -1        # n_entries below 3
    assert f(0.7, 65, 1, 1, buf, 256) == -1       # above 64
    assert f(0.7, 16, 4, 1, buf, 256) == -1       # degree 4
    assert f(0.05, 30, 1, 1, buf, 256) == -1      # r^29 / 2 below the FP32 normal range
    assert "underflows" in lib.aicdf_last_error().decode()
    assert f(0.05, 29, 1, 1, buf, 256) == 0
    assert f(0.7, 16, 1, 9, buf, 256) == -2       # bad dtype
    assert f(0.7, 16, 1, 1, buf, 31) == -6        # cap too small
    assert f(0.7, 16, 1, 1, None, 32) == -1
    h = C.c_void_p()
    assert lib.aicdf_table_geometric_create(0.7, 16, 1, 0, C.byref(h)) == -2  # F64 tables not stored
    assert lib.aicdf_table_geometric_create(0.99, 16, 1, 1, C.byref(h)) == -1
    assert not h.value
