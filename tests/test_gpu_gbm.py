"""GPU parity of the fused GBM MLMC level (Section 4) against the oracle's
per-path FP64 replay, plus the statistical pins of Section 4.1.

Per-path tolerances (FP32 path arithmetic against the FP64 replay on the
same uniforms; the oracle's approximate normals are evaluated in FP32 as in
the paper's Code 2, so both sides see the same Z~):
  EXACT, APPROX   |dP| <= 3e-7 N max(|P_f|, |P_c|, S0): one FP32 rounding of
                  relative size <= 1.5 eps32 per step, N = 2^l steps
  CORRECTION      |dD| <= 3e-7 N 0.05 S0 + 1e-5 |D| + 2.4e-7 S0: the difference
                  state e carries the same relative rounding (|e| <= 0.05 S0
                  for these tables), plus two FP32 roundings at scale S0 when
                  the path crosses the strike (the call's kink)
"""
import numpy as np
import pytest
import torch

import paper_2012_09715_amd as A
from oracle import gbm, tables
from oracle.dtypes import round_f32

pytestmark = pytest.mark.gpu
DEV = "cuda"

GBM = dict(S0=1.0, r=0.05, sigma=0.2, T=1.0, K=1.0, scheme=0, payoff=0)


def run_paths(params, level, n, kind, table, seed, offset=0):
    out = torch.zeros(n * 3, dtype=torch.float64, device=DEV)
    s = A.mlmc_level_gbm(params, level, n, kind, table, seed, offset, path_out=out)
    return s, out.cpu().numpy().reshape(n, 3)


@pytest.fixture(scope="module")
def lin16():
    return A.Table.dyadic(16, 1), ("dyadic_f32", round_f32(tables.dyadic_table(16, 1)))


@pytest.fixture(scope="module")
def const1024():
    return A.Table.const(1024, 0), ("const", round_f32(tables.const_table(1024)))


def check_paths(got, ref, kind, level, S0=1.0):
    N = 1 << level
    Y, Pf, Pc = ref
    if kind == 2:
        tol = 3e-7 * N * 0.05 * S0 + 1e-5 * np.abs(Y) + 2.4e-7 * S0
        assert np.all(np.abs(got[:, 0] - Y) <= tol), np.max(np.abs(got[:, 0] - Y) / tol)
        tolp = 3e-7 * N * np.maximum(np.maximum(np.abs(Pf), np.abs(Pc)), S0)
        assert np.all(np.abs(got[:, 1] - Pf) <= tolp)
        return
    scale = np.maximum(np.maximum(np.abs(Pf), np.abs(Pc)), S0)
    tol = 3e-7 * N * scale
    for j, r in enumerate((Y, Pf, Pc)):
        bad = np.abs(got[:, j] - r) > tol
        assert not bad.any(), (j, np.flatnonzero(bad)[:5], got[bad, j][:5], r[bad][:5])


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("payoff", [0, 1])
@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("level", [0, 1, 4])
def test_per_path_parity(lin16, scheme, payoff, kind, level):
    p = dict(GBM, scheme=scheme, payoff=payoff)
    n, seed, off = 1500, 1234 + level, 98765
    s, got = run_paths(p, level, n, kind, lin16[0], seed, off)
    ref = gbm.level_replay(p, level, kind, seed, off + np.arange(n), table=lin16[1])
    check_paths(got, ref, kind, level)
    assert s["n"] == n
    assert s["sum"][0] == pytest.approx(got[:, 0].sum(), rel=1e-12, abs=1e-12)
    assert s["sum"][1] == pytest.approx((got[:, 0] ** 2).sum(), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("kind", [1, 2])
def test_const_table_parity(const1024, kind):
    n, seed, level = 1000, 77, 3
    s, got = run_paths(GBM, level, n, kind, const1024[0], seed)
    ref = gbm.level_replay(GBM, level, kind, seed, np.arange(n), table=const1024[1])
    check_paths(got, ref, kind, level)


def test_level8_parity(lin16):
    n, seed, level = 300, 5, 8
    for kind in (0, 1, 2):
        _, got = run_paths(dict(GBM, payoff=1), level, n, kind, lin16[0], seed)
        ref = gbm.level_replay(dict(GBM, payoff=1), level, kind, seed, np.arange(n), table=lin16[1])
        check_paths(got, ref, kind, level)


def test_split_and_determinism(lin16):
    n = 5000
    for kind in (0, 1, 2):
        s, whole = run_paths(GBM, 3, n, kind, lin16[0], 9)
        _, a = run_paths(GBM, 3, 1234, kind, lin16[0], 9, 0)
        _, b = run_paths(GBM, 3, n - 1234, kind, lin16[0], 9, 1234)
        assert np.array_equal(whole, np.concatenate([a, b]))
        s2 = A.mlmc_level_gbm(GBM, 3, n, kind, lin16[0], 9)
        assert s["sum"] == s2["sum"] and s["sum_pf"] == s2["sum_pf"]


def test_sigma_zero(lin16):
    p = dict(GBM, sigma=0.0)
    for level in (0, 3, 7):
        N = 1 << level
        for kind in (0, 1, 2):
            _, got = run_paths(p, level, 256, kind, lin16[0], 1)
            assert np.allclose(got[:, 1], (1 + 0.05 / N) ** N, rtol=2e-7 * N)
            if kind == 2:
                assert np.all(got[:, 0] == 0.0)


def test_argument_errors(lin16):
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_level_gbm(GBM, 3, 100, 1, None, 0)
    with pytest.raises(A.AicdfError, match="ERANGE"):
        A.mlmc_level_gbm(GBM, 21, 100, 0, None, 0)
    with pytest.raises(A.AicdfError, match="EINVAL"):
        A.mlmc_level_gbm(GBM, 3, 100, 5, lin16[0], 0)
    s = A.mlmc_level_gbm(GBM, 3, 0, 0, None, 0)
    assert s["n"] == 0


def test_em_mean_closed_form(lin16):
    # E X_N = S0 (1 + r delta)^N for exact and any antisymmetric Z~ (5 sigma)
    n = 1 << 22
    for kind in (0, 1):
        for level in (0, 3, 6):
            s = A.mlmc_level_gbm(GBM, level, n, kind, lin16[0], 31 + level)
            m = s["sum_pf"] / n
            # sd(X_N) < 0.21 for sigma = 0.2, T = 1
            assert abs(m - gbm.em_mean(GBM, level)) < 5 * 0.21 / np.sqrt(n), (kind, level, m)


def test_telescoping_to_black_scholes(lin16):
    # sum_l E(P_l - P_(l-1)) = E(P_L) (Section 4) -> the call price, bias O(2^-L)
    p = dict(GBM, payoff=1)
    total, var = 0.0, 0.0
    for level in range(0, 9):
        n = 1 << (22 - min(level, 4))
        s = A.mlmc_level_gbm(p, level, n, 0, None, 100 + level)
        m = s["sum"][0] / n
        total += m
        var += (s["sum"][1] / n - m * m) / n
    bs = gbm.black_scholes_call(p)
    assert abs(total - bs) < 5 * np.sqrt(var) + 0.05 * 0.2 / 2 ** 8 * 4


def variance_drop(table, levels=(4, 6, 8), n=1 << 20):
    r = []
    for level in levels:
        s2 = A.mlmc_level_gbm(GBM, level, n, 0, None, 200 + level)
        s4 = A.mlmc_level_gbm(GBM, level, n, 2, table, 300 + level)
        v2 = s2["sum"][1] / n - (s2["sum"][0] / n) ** 2
        v4 = s4["sum"][1] / n - (s4["sum"][0] / n) ** 2
        r.append(np.log2(v4 / v2))
    return float(np.mean(r))


def test_variance_drop_table3(lin16, const1024):
    # Table 3 (EM, P = X): log2(V~/v^) about -13 (constant 1024), -14 (linear)
    d_lin = variance_drop(lin16[0])
    d_const = variance_drop(const1024[0])
    assert -15.5 < d_lin < -12.5, d_lin
    assert -14.5 < d_const < -11.5, d_const
    cubic = A.Table.dyadic(16, 3)
    d_cub = variance_drop(cubic)
    assert d_cub < d_lin - 4, d_cub


def test_nested_identity_on_means(lin16):
    # E(Y~) + E(D) = E(Y^) on every level (the nested decomposition of Section 4)
    n = 1 << 22
    for level in (1, 5):
        e = A.mlmc_level_gbm(GBM, level, n, 0, None, 400 + level)
        a = A.mlmc_level_gbm(GBM, level, n, 1, lin16[0], 500 + level)
        c = A.mlmc_level_gbm(GBM, level, n, 2, lin16[0], 600 + level)
        mean = lambda s: s["sum"][0] / n
        var = lambda s: s["sum"][1] / n - mean(s) ** 2
        se = np.sqrt((var(e) + var(a) + var(c)) / n)
        assert abs(mean(a) + mean(c) - mean(e)) < 5 * se


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("scheme", [0, 1])
def test_wave_per_path_launch(lin16, kind, scheme):
    # calls of <= 8192 paths with 2^l >= 128 steps run one path per wavefront
    # (products of step maps, reduced over the lanes): against the oracle, bit
    # reproducible within that launch shape, and equal to one path per thread
    # to FP32 rounding
    p = dict(GBM, scheme=scheme, payoff=1)
    level, seed = 9, 404 + kind
    _, few = run_paths(p, level, 200, kind, lin16[0], seed, 1000)
    ref = gbm.level_replay(p, level, kind, seed, 1000 + np.arange(200), table=lin16[1])
    check_paths(few, ref, kind, level)
    _, a = run_paths(p, level, 120, kind, lin16[0], seed, 1000)
    assert np.array_equal(a, few[:120])
    _, many = run_paths(p, level, 9000, kind, lin16[0], seed, 0)
    check_paths(many[1000:1200], ref, kind, level)


def test_rademacher_table_and_variance():
    # Rademacher variables as the 2-interval table {-1, +1} (Section 1, Table
    # 3's first row): the transform gives sign(u - 1/2); the fused levels
    # match the oracle, and the four-way variance drops only by about 2^-1
    # against the two-way one (Table 3: log2 ratio -1), the reason the paper
    # calls them too crude for nested MLMC
    rad = A.Table.rademacher()
    u = torch.tensor([0.1, 0.4999, 0.5, 0.9, 1e-9, 1 - 2 ** -24], dtype=torch.float32, device=DEV)
    z = A.approx_icdf_const(rad, u).cpu().numpy()
    assert np.array_equal(z, [-1, -1, 1, 1, -1, 1])
    tab = ("const", np.array([-1.0, 1.0]))
    for kind in (1, 2):
        _, got = run_paths(GBM, 4, 500, kind, rad, 61 + kind)
        ref = gbm.level_replay(GBM, 4, kind, 61 + kind, np.arange(500), table=tab)
        # |X^ - X~| reaches ~0.3 S0 with +-1 normals: the FP32 rounding bound
        # of the difference state is that of a full path
        tol = 3e-7 * 16 * np.maximum(np.abs(ref[1]), 1.0) + 2.4e-7
        for j in range(3):
            assert np.all(np.abs(got[:, j] - ref[j]) <= tol), (kind, j)
    n = 1 << 20
    for level in (2, 4, 6):
        s2 = A.mlmc_level_gbm(GBM, level, n, 0, None, 70 + level)
        s4 = A.mlmc_level_gbm(GBM, level, n, 2, rad, 80 + level)
        v = lambda s: s["sum"][1] / n - (s["sum"][0] / n) ** 2
        r = np.log2(v(s4) / v(s2))
        assert -2.0 < r < -0.3, (level, r)


@pytest.mark.parametrize("scheme", [0, 1])
def test_config_size_sampled(lin16, scheme):
    # a level of the benchmark's configuration: 10^6 paths at level 8 (one
    # path per thread, the full grid), checked on paths sampled across the range
    n, level, seed = 1_000_000, 8, 77
    p = dict(GBM, scheme=scheme, payoff=1)
    pick = np.unique(np.concatenate([np.random.default_rng(scheme).integers(0, n, 60), [0, 1, n - 2, n - 1]]))
    for kind in (0, 1, 2):
        s, got = run_paths(p, level, n, kind, lin16[0], seed)
        ref = gbm.level_replay(p, level, kind, seed, pick, table=lin16[1])
        check_paths(got[pick], ref, kind, level)
        assert s["n"] == n


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_level10_milstein_wave_shape(lin16, kind):
    # the finest level of the large fused run (1024 Milstein steps), a few
    # paths in the one-path-per-wavefront shape, against the oracle's replay
    p = dict(GBM, scheme=1, payoff=1)
    level, seed, off = 10, 1010 + kind, 5_000_000
    _, got = run_paths(p, level, 6, kind, lin16[0], seed, off)
    ref = gbm.level_replay(p, level, kind, seed, off + np.arange(6), table=lin16[1])
    check_paths(got, ref, kind, level)


@pytest.mark.parametrize("level", [2, 3, 5, 7])
def test_group_shapes(lin16, level):
    # calls with paths x G <= 2^19 run one path per group of G = min(64, 2^l/2)
    # lanes: against the oracle, and against one path per thread (a call too
    # large for groups) to FP32 rounding
    p = dict(GBM, scheme=1, payoff=1)
    G = min(64, (1 << level) // 2)
    for kind in (0, 1, 2):
        seed = 300 + 10 * level + kind
        _, few = run_paths(p, level, 100, kind, lin16[0], seed, 0)
        ref = gbm.level_replay(p, level, kind, seed, np.arange(100), table=lin16[1])
        check_paths(few, ref, kind, level)
        _, dense = run_paths(p, level, (1 << 19) // G + 1, kind, lin16[0], seed, 0)
        check_paths(dense[:100], ref, kind, level)
