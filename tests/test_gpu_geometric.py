"""GPU parity of the geometric-interval tables (Theorem 2.5 with a general
decay rate r) against the oracle: the streaming transform, its row index, and
the fused GBM levels that draw their approximate normals from such a table.

Tolerances
  row index     bit-exact (uint32): both sides compare the FP32 input with
                the same FP32 thresholds B_e
  F32 output    per element, with eps = 2^-24, c the stored row and
                s = t / B_e:
                  4 (d + 1) eps sum_j |c_j| s^j      (FP32 Horner with FMAs)
                + 3 eps s |p'(s)|                    (s = t * fl(1/B_e) in FP32)
                + sum_j ulp32(c_j) s^j               (the library's and the
                  oracle's FP64 fits agree to ~1e-11, so their FP32 roundings
                  may differ by one ulp)
  16-bit out    one ulp of the output dtype on top of the F32 bound
  GBM levels    as for the dyadic tables (FP32 path arithmetic against the
                FP64 replay on the same uniforms)
"""
import math

import numpy as np
import pytest
import torch

import paper_2012_09715_amd as A
from oracle import gbm, tables
from oracle.dtypes import ROUND, round_f32, ulp
from oracle.normal import Phi_inv
from tests.inputs import edge_uniforms, random_u24, random_uniforms

pytestmark = pytest.mark.gpu
DEV = "cuda"
TORCH_DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
EPS = 2.0 ** -24

_cache = {}


def oracle_table(r, T, d, coef="f32"):
    key = (r, T, d, coef)
    if key not in _cache:
        _cache[key] = ROUND[coef](tables.geometric_table(r, T, d))
    return _cache[key]


def threshold_inputs(r, T):
    B = tables.geometric_thresholds(r, T).astype(np.float32)
    v = []
    for b in B:
        for x in (b, np.nextafter(b, np.float32(0)), np.nextafter(b, np.float32(1))):
            v += [x, np.float32(1) - x]
    return np.array(v, dtype=np.float32)


def inputs(r, T, n, seed):
    return np.concatenate([edge_uniforms(np.float32), threshold_inputs(r, T),
                           random_uniforms(n, seed, np.float32)])


def bound(tab, r, u):
    """Per-element tolerance of the F32 transform (module docstring)."""
    u = u.astype(np.float64)
    T, d1 = tab.shape
    t = np.where(u < 0.5, u, 1.0 - u)
    e = tables.geometric_row(t, r, T)
    B = tables.geometric_thresholds(r, T)
    s = np.abs(t / B[e])
    c = tab[e]
    absum = sum(np.abs(c[:, j]) * s ** j for j in range(d1))
    deriv = np.abs(sum(j * c[:, j] * s ** (j - 1) for j in range(1, d1))) if d1 > 1 else 0.0
    sp = np.spacing(np.abs(c).astype(np.float32)).astype(np.float64)
    coef = sum(sp[:, j] * s ** j for j in range(d1))
    return 4 * d1 * EPS * absum + 3 * EPS * s * deriv + coef


def check(z, zo, tol, out):
    nan = np.isnan(zo)
    assert np.array_equal(np.isnan(z), nan)
    z, zo, tol = z[~nan], zo[~nan], tol[~nan]
    if out != "f32":
        tol = tol + ulp(ROUND[out](zo), out) * 1.0001
    bad = np.abs(z - zo) > tol
    assert not bad.any(), (np.flatnonzero(bad)[:5], z[bad][:5], zo[bad][:5], tol[bad][:5])


def to_np(z):
    return z.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("r,T", [(0.3, 40), (0.7, 64), (0.95, 64), (0.05, 29)])
@pytest.mark.parametrize("d", [0, 1, 3])
def test_geometric_transform_parity(r, T, d):
    tab = A.Table.geometric(r, T, d)
    ot = oracle_table(r, T, d)
    u = inputs(r, T, 100_003, seed=int(r * 100) + d)
    ug = torch.from_numpy(u).to(DEV)
    idx = A.approx_icdf_index(tab, ug).cpu().numpy().astype(np.int64)
    t = np.where(u < 0.5, u.astype(np.float64), 1.0 - u.astype(np.float64))
    assert np.array_equal(idx, tables.geometric_row(t, r, T))
    zo = tables.geometric_transform(ot, r, u.astype(np.float64))
    tol = bound(ot, r, u)
    for out in ("f32", "f16", "bf16"):
        z = to_np(A.approx_icdf_linear(tab, ug, out_dtype=TORCH_DT[out]))
        check(z, zo, tol, out)


@pytest.mark.parametrize("coef", ["f16", "bf16"])
def test_geometric_16bit_coefficients(coef):
    r, T, d = 0.7, 48, 3
    tab = A.Table.geometric(r, T, d, TORCH_DT[coef])
    ot = ROUND[coef](A.geometric_host_coeffs(r, T, d, torch.float64).numpy())
    assert np.array_equal(tab.coeffs().numpy(), ot)
    u = inputs(r, T, 50_000, seed=3)
    zo = tables.geometric_transform(ot, r, u.astype(np.float64))
    z = to_np(A.approx_icdf_linear(tab, torch.from_numpy(u).to(DEV)))
    check(z, zo, bound(ot, r, u), "f32")


def test_geometric_half_rate_matches_dyadic():
    # r = 1/2: the same rows as the exponent read of Algorithm 1 and, up to the
    # last-ulp differences of the two FP64 fits, the same values
    for d in (1, 3):
        g, y = A.Table.geometric(0.5, 16, d), A.Table.dyadic(16, d)
        un = inputs(0.5, 16, 200_000, seed=11)
        u = torch.from_numpy(un).to(DEV)
        num = torch.from_numpy(~np.isnan(un)).to(DEV)  # a NaN has no row; the two conventions differ
        assert torch.equal(A.approx_icdf_index(g, u)[num], A.approx_icdf_index(y, u)[num])
        zg, zy = to_np(A.approx_icdf_linear(g, u)), to_np(A.approx_icdf_linear(y, u))
        ok = ~np.isnan(zy)
        assert np.array_equal(np.isnan(zg), ~ok)
        assert np.all(np.abs(zg[ok] - zy[ok]) <= 2e-6 * np.maximum(1.0, np.abs(zy[ok])))


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4095, 4097, (1 << 20) + 13])
def test_geometric_sizes(n):
    r, T, d = 0.8, 64, 1
    tab = A.Table.geometric(r, T, d)
    ot = oracle_table(r, T, d)
    u = random_uniforms(n, seed=n % 1000 + 1, dtype=np.float32)
    ug = torch.from_numpy(u).to(DEV)
    z = to_np(A.approx_icdf_linear(tab, ug))
    idx = A.approx_icdf_index(tab, ug).cpu().numpy().astype(np.int64)
    assert z.shape == (n,) and idx.shape == (n,)
    if n:
        t = np.where(u < 0.5, u.astype(np.float64), 1.0 - u.astype(np.float64))
        assert np.array_equal(idx, tables.geometric_row(t, r, T))
        check(z, tables.geometric_transform(ot, r, u.astype(np.float64)), bound(ot, r, u), "f32")


def test_geometric_large_sampled():
    # 2^26 + 5 inputs in the benchmark's launch shape, checked on a sample
    r, T, d = 0.7, 64, 3
    n = (1 << 26) + 5
    tab = A.Table.geometric(r, T, d)
    ot = oracle_table(r, T, d)
    u = torch.empty(n, dtype=torch.float32, device=DEV)
    A.uniform_fill(u, seed=99)
    z = A.approx_icdf_linear(tab, u)
    pick = np.unique(np.concatenate([np.random.default_rng(1).integers(0, n, 50_000), [0, n - 5, n - 1]]))
    us = u[torch.from_numpy(pick).to(DEV)].cpu().numpy()
    zs = to_np(z[torch.from_numpy(pick).to(DEV)])
    check(zs, tables.geometric_transform(ot, r, us.astype(np.float64)), bound(ot, r, us), "f32")


def test_geometric_rmse_on_device():
    # the device transform's RMSE against the exact inverse on 2^24 uniforms
    # agrees with the oracle's L2 error (projection identity) to MC accuracy
    n = 1 << 24
    u = torch.empty(n, dtype=torch.float32, device=DEV)
    A.uniform_fill(u, seed=5)
    zx = A.exact_icdf(u, out_dtype=torch.float64)
    for r, T, d in ((0.7, 64, 1), (0.8, 64, 1), (0.6, 64, 3)):
        z = A.approx_icdf_linear(A.Table.geometric(r, T, d), u).double()
        got = math.sqrt(float(((z - zx) ** 2).mean()))
        want = tables.geometric_l2_error(tables.geometric_table(r, T, d), r)
        assert abs(got / want - 1) < 0.03, (r, d, got, want)


def test_geometric_errors():
    tab = A.Table.geometric(0.7, 16, 1)
    u64 = torch.rand(10, dtype=torch.float64, device=DEV)
    with pytest.raises(A.AicdfError, match="EDTYPE"):
        A.approx_icdf_linear(tab, u64)
    with pytest.raises(A.AicdfError, match="EDTYPE"):
        A.approx_icdf_index(tab, u64)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.approx_icdf_const(tab, u64.float())
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.Table.geometric(0.99, 16, 1)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.Table.geometric(0.05, 40, 1)
    with pytest.raises(A.AicdfError, match="EDTYPE"):
        A.Table.geometric(0.7, 16, 1, torch.float64)


# ---------------------------------------------------------------- fused GBM levels
GBM = dict(S0=1.0, r=0.05, sigma=0.2, T=1.0, K=1.0, scheme=0, payoff=0)


def check_paths(got, ref, kind, level, S0=1.0):
    N = 1 << level
    Y, Pf, Pc = ref
    if kind == 2:
        tol = 3e-7 * N * 0.05 * S0 + 1e-5 * np.abs(Y) + 2.4e-7 * S0
        assert np.all(np.abs(got[:, 0] - Y) <= tol), np.max(np.abs(got[:, 0] - Y) / tol)
        assert np.all(np.abs(got[:, 1] - Pf) <= 3e-7 * N * np.maximum(np.abs(Pf), S0))
        return
    scale = np.maximum(np.maximum(np.abs(Pf), np.abs(Pc)), S0)
    for j, r in enumerate((Y, Pf, Pc)):
        assert np.all(np.abs(got[:, j] - r) <= 3e-7 * N * scale), j


@pytest.mark.parametrize("scheme,payoff", [(0, 0), (1, 1)])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("level,n", [(0, 300), (4, 300), (8, 200)])
def test_gbm_level_with_geometric_table(scheme, payoff, kind, level, n):
    # level 8 with 200 paths runs one path per wavefront
    r, T, d = 0.75, 48, 3
    tab = A.Table.geometric(r, T, d)
    ot = round_f32(tables.geometric_table(r, T, d))
    p = dict(GBM, scheme=scheme, payoff=payoff)
    seed = 40 + level + 10 * kind
    out = torch.zeros(n * 3, dtype=torch.float64, device=DEV)
    A.mlmc_level_gbm(p, level, n, kind, tab, seed, 0, path_out=out)
    got = out.cpu().numpy().reshape(n, 3)
    ref = gbm.level_replay(p, level, kind, seed, np.arange(n), table=("geometric", (ot, r)))
    check_paths(got, ref, kind, level)


def test_gbm_correction_variance_follows_l2_error():
    # the nested correction's variance falls with the L2 error of the
    # approximation: dyadic linear (6.4e-3), geometric linear r = 0.8
    # (6.6e-4), geometric cubic r = 0.7 (7.1e-6).  The variance also carries
    # the u53-versus-u24 quantisation of the correction kind's draws, whose
    # tail samples make the estimate heavy-tailed, so only the order and a
    # loose size of the drop are checked (the FP64 replay of 10^5 paths gives
    # a ratio of 2.7e-6 between the last and the first).
    n, level = 1 << 20, 4

    def var(tab, seed):
        s = A.mlmc_level_gbm(GBM, level, n, 2, tab, seed)
        m = s["sum"][0] / n
        return s["sum"][1] / n - m * m

    v = [var(A.Table.dyadic(16, 1), 2), var(A.Table.geometric(0.8, 64, 1), 3), var(A.Table.geometric(0.7, 64, 3), 1)]
    assert v[0] > v[1] > v[2], v
    assert v[2] / v[0] < 3e-5, v
