"""GPU parity of the streaming transforms against the oracle (Code 1,
Algorithm 1, Section 3.1's exact inverse) and of the uniform fill.

Tolerances
  indices             bit-exact (uint32)
  dyadic, F32 output  |z - z_oracle| <= 1e-6 max(1, |z_oracle|), z_oracle the
                      FP64 evaluation on the oracle's own FP32-rounded table
  16-bit outputs      within 1 ulp of the output dtype of the oracle's value
                      rounded to that dtype, plus the FP32 evaluation bound
                      above (the FP32 result near z = 0 carries an absolute
                      error ~1e-7 that a fine 16-bit ulp can resolve)
  F64 input           |z - z_oracle| <= 1e-14 max(1, |z|) + sum_j ulp32(c_j) s^j:
                      the library's and the oracle's FP64 fits agree to ~1e-9,
                      so their FP32-rounded coefficients may differ by one ulp
  constant tables     within 1 ulp of the coarser of output and coefficient
                      dtype of the oracle constant (FP64 constants: 4 N eps
                      absolute, the oracle's closed form cancels)
  exact Phi^-1 (FP64) |z - z_oracle| <= 4e-15 max(1, |z_oracle|)
  uniforms            bit-exact
"""
import numpy as np
import pytest
import torch

import paper_2012_09715_amd as A
from oracle import rng as orng
from oracle import tables, transform
from oracle.dtypes import ROUND, ulp
from oracle.normal import Phi_inv
from tests.inputs import edge_uniforms, random_u24, random_uniforms

pytestmark = pytest.mark.gpu

DEV = "cuda"
TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
NP_IN = {"f32": np.float32, "f64": np.float64}

_dyadic_cache = {}


def oracle_dyadic(T, d, coef):
    key = (T, d, coef)
    if key not in _dyadic_cache:
        _dyadic_cache[key] = ROUND[coef](tables.dyadic_table(T, d))
    return _dyadic_cache[key]


def to_np(z):
    return z.float().cpu().numpy().astype(np.float64) if z.dtype in (torch.float16, torch.bfloat16) else \
        z.cpu().numpy().astype(np.float64)


def inputs(in_dt, n, seed):
    u = np.concatenate([edge_uniforms(NP_IN[in_dt]), random_uniforms(n, seed, NP_IN[in_dt])])
    return u


def check_values(z, ref, out_dt, tol_rel=1e-6, slack=None):
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(z), nan)
    z, ref = z[~nan], ref[~nan]
    extra = 0.0 if slack is None else slack[~nan]
    if out_dt in ("f32", "f64"):
        err = np.abs(z - ref)
        bad = err > tol_rel * np.maximum(1.0, np.abs(ref)) + extra
        assert not bad.any(), (np.flatnonzero(bad)[:5], z[bad][:5], ref[bad][:5])
    else:
        r = ROUND[out_dt](ref)
        bad = np.abs(z - r) > ulp(r, out_dt) * 1.0001 + 1e-6 * np.maximum(1.0, np.abs(ref))
        assert not bad.any(), (z[bad][:5], r[bad][:5])


def coef_slack(tab, u):
    """sum_j ulp32(c_j) s^j on the row the oracle selects for each u."""
    e, p, ur = transform.dyadic_index(tab.shape[0], u)
    s = np.ldexp(ur, e + 1)
    c = tab[e]
    sp = np.spacing(np.abs(c).astype(np.float32)).astype(np.float64)
    return sum(sp[:, j] * np.abs(s) ** j for j in range(tab.shape[1]))


@pytest.mark.parametrize("T", [8, 16, 32])
@pytest.mark.parametrize("d", [0, 1, 2, 3])
@pytest.mark.parametrize("coef", ["f32", "f16", "bf16"])
def test_dyadic_f32_input(T, d, coef):
    tab = A.Table.dyadic(T, d, TORCH_DT[coef])
    ot = oracle_dyadic(T, d, coef)
    u = inputs("f32", 100_003, seed=T * 10 + d)
    ug = torch.from_numpy(u).to(DEV)
    idx = A.approx_icdf_index(tab, ug).cpu().numpy().astype(np.int64)
    zo, eo = transform.dyadic_transform(ot, u.astype(np.float64))
    assert np.array_equal(idx, eo)
    for out in ("f32", "f16", "bf16"):
        z = to_np(A.approx_icdf_linear(tab, ug, out_dtype=TORCH_DT[out]))
        check_values(z, zo, out)


@pytest.mark.parametrize("T,d", [(16, 1), (16, 3), (32, 3), (8, 1)])
def test_dyadic_f64_input(T, d):
    tab = A.Table.dyadic(T, d, torch.float32)
    ot = oracle_dyadic(T, d, "f32")
    u = inputs("f64", 100_001, seed=7)
    ug = torch.from_numpy(u).to(DEV)
    idx = A.approx_icdf_index(tab, ug).cpu().numpy().astype(np.int64)
    zo, eo = transform.dyadic_transform(ot, u)
    assert np.array_equal(idx, eo)
    slack = coef_slack(ot, u)
    z64 = to_np(A.approx_icdf_linear(tab, ug, out_dtype=torch.float64))
    check_values(z64, zo, "f64", tol_rel=1e-14, slack=slack)
    z32 = to_np(A.approx_icdf_linear(tab, ug, out_dtype=torch.float32))
    check_values(z32, zo, "f32", tol_rel=1.2e-7, slack=slack)


def test_dyadic_special_values():
    tab = A.Table.dyadic(16, 1, torch.float32)
    u = torch.tensor([0.5, 0.0, 1.0, float("nan")], device=DEV)
    z = A.approx_icdf_linear(tab, u).cpu().numpy()
    c = tab.coeffs().numpy()
    assert z[0] == 0.0
    assert z[1] == np.float32(c[15, 0]) and z[2] == -np.float32(c[15, 0])
    assert np.isnan(z[3])


def test_dyadic_antisymmetry_bitwise():
    tab = A.Table.dyadic(16, 3, torch.float32)
    u = random_u24(1 << 20, 5)
    a = A.approx_icdf_linear(tab, torch.from_numpy(u).to(DEV)).cpu().numpy()
    b = A.approx_icdf_linear(tab, torch.from_numpy((1 - u.astype(np.float64)).astype(np.float32)).to(DEV)).cpu().numpy()
    assert np.array_equal(a, -b)


@pytest.mark.parametrize("N", [2, 16, 1024, 65536])
@pytest.mark.parametrize("construction", [0, 1, 2])
def test_const_tables(N, construction):
    for coef in ("f32", "f64"):
        tab = A.Table.const(N, construction, TORCH_DT[coef])
        Q = tables.const_table(N, "ECI"[construction])
        for in_dt in ("f32", "f64"):
            if coef == "f64" and in_dt == "f32":
                continue
            u = inputs(in_dt, 50_000, seed=N + construction)
            ug = torch.from_numpy(u).to(DEV)
            idx = A.approx_icdf_index(tab, ug).cpu().numpy().astype(np.int64)
            m = transform.const_index(N, u.astype(np.float64))
            assert np.array_equal(idx, m)
            ref = Q[m]
            outs = ("f32", "f16", "bf16") if in_dt == "f32" else ("f32", "f64")
            for out in outs:
                z = to_np(A.approx_icdf_const(tab, ug, out_dtype=TORCH_DT[out]))
                r = ROUND[out](ROUND[coef](ref)) if out != "f64" else ROUND[coef](ref)
                # one ulp of the coarser of output and coefficient dtype: the two
                # FP64 constructions may round to neighbouring FP32 constants
                # FP64 constants: the oracle's closed form subtracts two
                # densities and loses ~N eps absolute (N = 65536: ~6e-11)
                tol = (np.maximum(ulp(r, out), ulp(r, coef)) * 1.0001 if coef != "f64"
                       else 4 * N * 2.2e-16 + 1e-12 * np.abs(r) + ulp(r, out))
                bad = np.abs(z - r) > tol
                assert not bad.any(), (N, construction, coef, in_dt, out, z[bad][:4], r[bad][:4])


def test_exact_icdf_f64():
    u = np.concatenate([edge_uniforms(np.float64), random_uniforms(200_000, 3, np.float64)])
    u = u[(np.isnan(u)) | (np.minimum(u, 1 - u) >= 1e-300) | (u == 0) | (u == 1)]
    zo = Phi_inv(u)
    z = A.exact_icdf(torch.from_numpy(u).to(DEV)).cpu().numpy()
    fin = np.isfinite(zo)
    assert np.array_equal(np.isnan(z), np.isnan(zo))
    assert np.array_equal(z[np.isinf(zo)], zo[np.isinf(zo)])
    err = np.abs(z[fin] - zo[fin]) / np.maximum(1.0, np.abs(zo[fin]))
    assert err.max() <= 4e-15, err.max()


def test_exact_icdf_f32_in_out():
    u = np.concatenate([edge_uniforms(np.float32), random_uniforms(100_000, 4, np.float32)])
    ug = torch.from_numpy(u).to(DEV)
    zo = Phi_inv(u.astype(np.float64))
    z64 = A.exact_icdf(ug).cpu().numpy()
    z32 = A.exact_icdf(ug, out_dtype=torch.float32).cpu().numpy().astype(np.float64)
    fin = np.isfinite(zo)
    assert np.all(np.abs(z64[fin] - zo[fin]) <= 4e-15 * np.maximum(1, np.abs(zo[fin])))
    assert np.all(np.abs(z32[fin] - zo[fin]) <= ulp(zo[fin], "f32"))


@pytest.mark.parametrize("n,offset", [(1 << 20, 0), (1000, 3), (7, 1), (4097, 4096 + 2), (1, 0)])
def test_uniform_fill_bit_exact(n, offset):
    for seed, sid in ((20201217, 0), (1, 5), (2 ** 63 + 12345, 2 ** 40 + 7)):
        u = torch.empty(n, dtype=torch.float32, device=DEV)
        A.uniform_fill(u, seed, sid, offset)
        assert np.array_equal(u.cpu().numpy(), orng.uniform_fill_f32(seed, sid, offset, n))
        v = torch.empty(n, dtype=torch.float64, device=DEV)
        A.uniform_fill(v, seed, sid, offset)
        assert np.array_equal(v.cpu().numpy(), orng.uniform_fill_f64(seed, sid, offset, n))


def test_uniform_fill_unaligned_view():
    base = torch.empty(1001, dtype=torch.float32, device=DEV)
    A.uniform_fill(base[1:], 9, 0, 0)
    assert np.array_equal(base[1:].cpu().numpy(), orng.uniform_fill_f32(9, 0, 0, 1000))


@pytest.mark.parametrize("n", [0, 1, 5, 4095, 4096, 4097, 3 * 4096 + 17])
def test_ragged_and_unaligned(n):
    tab = A.Table.dyadic(16, 1, torch.float32)
    ot = oracle_dyadic(16, 1, "f32")
    base = torch.from_numpy(random_uniforms(n + 1, n, np.float32)).to(DEV)
    for u in (base[:n], base[1:]):
        out = torch.full((n + 1,), 7.0, device=DEV)
        z = A.approx_icdf_linear(tab, u, z=out[:n])
        zo, _ = transform.dyadic_transform(ot, u.cpu().numpy().astype(np.float64))
        check_values(to_np(z), zo, "f32")
        assert out[n].item() == 7.0  # nothing written past the end


def test_alias_rejected():
    tab = A.Table.dyadic(16, 1, torch.float32)
    u = torch.rand(1000, device=DEV)
    with pytest.raises(A.AicdfError, match="EALIAS"):
        A.approx_icdf_linear(tab, u, z=u)


def test_bw_probe_copy_and_write():
    src = torch.arange(1 << 20, dtype=torch.float32, device=DEV)
    dst = torch.zeros_like(src)
    A.bw_probe(0, src, dst)
    assert torch.equal(src, dst)
    A.bw_probe(2, None, dst)
    torch.cuda.synchronize()


def test_full_size_u24_stream_sampled():
    """2^30 device uniforms -> linear-16 FP32, the benchmark's launch; outputs
    checked on a random sample of 2^17 positions and by exact symmetry counts."""
    n = 1 << 30
    tab = A.Table.dyadic(16, 1, torch.float32)
    ot = oracle_dyadic(16, 1, "f32")
    u = torch.empty(n, dtype=torch.float32, device=DEV)
    A.uniform_fill(u, 20201217, 3, 0)
    z = A.approx_icdf_linear(tab, u)
    pos = torch.from_numpy(np.random.default_rng(0).integers(0, n, 1 << 17)).to(DEV)
    us = u[pos].cpu().numpy()
    p0 = int(pos[0].item())
    assert np.array_equal(u[p0:p0 + 64].cpu().numpy(), orng.uniform_fill_f32(20201217, 3, p0, 64))
    zo, _ = transform.dyadic_transform(ot, us.astype(np.float64))
    check_values(z[pos].cpu().numpy().astype(np.float64), zo, "f32")
    # the u24 grid is symmetric, so the mean of z is ~0 (antisymmetric table)
    m = z.double().mean().item()
    assert abs(m) < 5.0 / np.sqrt(n) * 1.0
    del u, z
    torch.cuda.empty_cache()


def test_half_outputs_are_rne_of_the_f32_output():
    # the F16/BF16 outputs are the FP32 result rounded to nearest even (the
    # BF16 one by the hardware conversion): checked bit for bit against the
    # oracle's integer RNE on about 2^20 values, ties included
    from oracle.dtypes import bf16_bits_from_f64
    tab = A.Table.dyadic(16, 3)
    u = torch.from_numpy(inputs("f32", 1 << 20, seed=99)).to(DEV)
    z32 = A.approx_icdf_linear(tab, u).cpu().numpy()
    zb = A.approx_icdf_linear(tab, u, out_dtype=torch.bfloat16).view(torch.int16).cpu().numpy().view(np.uint16)
    zh = A.approx_icdf_linear(tab, u, out_dtype=torch.float16).cpu().numpy()
    ok = np.isfinite(z32) & ((z32 == 0) | (np.abs(z32) >= 2.0 ** -126))
    assert ok.sum() > (1 << 20) - 16
    want = bf16_bits_from_f64(z32[ok].astype(np.float64))
    assert np.array_equal(zb[ok], want)
    assert np.sum((z32[ok].view(np.uint32) & 0xFFFF) == 0x8000) >= 1  # a tie was exercised
    assert np.array_equal(zh[ok].view(np.uint16), z32[ok].astype(np.float64).astype(np.float16).view(np.uint16))
    assert np.array_equal((zb & 0x7FFF) > 0x7F80, np.isnan(z32))
