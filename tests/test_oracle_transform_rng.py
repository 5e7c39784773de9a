"""Pins of the oracle's transforms (Code 1, Algorithm 1, Table 1) and RNG."""
import numpy as np
import pytest
from scipy import stats

from oracle import rng, tables, transform
from oracle.dtypes import bf16_bits_from_f64, bf16_bits_to_f64, round_bf16
from tests.conftest import read_golden


# ---------------------------------------------------------------- indices
def test_dyadic_index_table1():
    # Table 1: index n <-> [2^-(n+1), 2^-n); the capped entry N <-> (0, 2^-N)
    T = 16
    for n in range(1, T - 1):
        lo, hi = 2.0 ** -(n + 1), 2.0 ** -n
        u = np.array([lo, np.nextafter(hi, 0.0), 0.5 * (lo + hi)])
        e, p, ur = transform.dyadic_index(T, u)
        assert np.all(e == n) and np.all(p)
    e, _, _ = transform.dyadic_index(T, np.array([np.nextafter(2.0 ** -(T - 1), 0), 2.0 ** -15 * 0.999, 1e-300, 5e-324, 0.0, 2.0 ** -(T - 1)]))
    assert list(e) == [T - 1] * 5 + [T - 2]


def test_dyadic_index_half_and_reflection():
    e, p, ur = transform.dyadic_index(16, np.array([0.5, 0.75, 1.0 - 2.0 ** -20, 1.0]))
    assert list(e) == [0, 1, 15, 15]
    assert list(p) == [False, False, False, False]
    assert ur[1] == 0.25


def test_dyadic_values_half_zero_and_antisymmetry():
    tab = tables.dyadic_table(16, 3)
    z, _ = transform.dyadic_transform(tab, np.array([0.5]))
    assert z[0] == 0.0
    rng_ = np.random.default_rng(3)
    u = rng_.random(10000)
    v = 1.0 - u
    ok = (1.0 - v) == u
    assert np.array_equal(transform.dyadic_transform(tab, v)[0][ok], -transform.dyadic_transform(tab, u)[0][ok])


def test_dyadic_value_matches_u_monomials():
    tab = tables.dyadic_table(16, 1)
    u = np.array([0.3, 0.1, 1e-3, 1e-6])
    z, e = transform.dyadic_transform(tab, u)
    for i in range(len(u)):
        a = tables.to_u_monomials(tab[e[i]], int(e[i]))
        assert z[i] == pytest.approx(a[0] + a[1] * u[i], rel=1e-12)


def test_const_index_clamp_and_edges():
    N = 1024
    u = np.array([0.0, 1.0 / N, np.nextafter(1.0 / N, 0), 0.5, 1.0, np.nan, -0.5, 2.0])
    assert list(transform.const_index(N, u)) == [0, 1, 0, 512, N - 1, 0, 0, N - 1]


def test_dtype_rounding_bf16():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -3.37365053, 1.0 + 2.0 ** -8 + 2.0 ** -30])
    r = round_bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0  # tie to even
    assert r[2] == 1.0 + 2 * 2.0 ** -7  # tie to even upward
    assert r[4] == 1.0 + 2.0 ** -7      # above the tie rounds up
    assert bf16_bits_from_f64(np.array([-2.0]))[0] == 0xC000
    assert bf16_bits_to_f64(np.array([0x3F80], dtype=np.uint16))[0] == 1.0


# ---------------------------------------------------------------- RNG
def test_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt"):
        vals = [int(v, 16) for v in row]
        out = rng.philox4x32_10(np.array(vals[:4], dtype=np.uint32), np.array(vals[4:6], dtype=np.uint32))
        assert [int(v) for v in out] == vals[6:]


def test_u24_grid():
    w = np.array([0, 0xFFFFFFFF, 0x80000000, 511, 512], dtype=np.uint32)
    u = rng.u24_from_word(w)
    assert u.dtype == np.float32
    assert u[0] == 2.0 ** -24 and u[1] == 1.0 - 2.0 ** -24 and u[2] == 0.5 + 2.0 ** -24
    assert u[3] == u[0] and u[4] == 3 * 2.0 ** -24
    allw = (np.arange(1 << 23, dtype=np.uint32) << np.uint32(9))
    g = rng.u24_from_word(allw).astype(np.float64)
    assert np.array_equal(np.sort(1.0 - g), g)  # symmetric about 1/2


def test_u53_formula_and_top_value():
    u = rng.u53_from_words(np.array([0, 0xFFFFFFFF, 0x80000000], dtype=np.uint32),
                           np.array([0, 0xFFFFFFFF, 0], dtype=np.uint32))
    assert u[0] == 2.0 ** -54
    assert u[1] == 1.0 - 2.0 ** -53  # (2^53 - 1 + 0.5) 2^-53 rounds to 1 -> mapped below 1
    assert u[2] == 0.5  # k = 2^52: 2^52 + 0.5 ties to even = 2^52
    assert np.all(u < 1.0) and np.all(u > 0.0)


def test_fill_layout_offsets():
    a = rng.uniform_fill_f32(7, 3, 0, 1000)
    b = rng.uniform_fill_f32(7, 3, 123, 500)
    assert np.array_equal(a[123:623], b)
    a = rng.uniform_fill_f64(7, 3, 0, 1000)
    b = rng.uniform_fill_f64(7, 3, 77, 600)
    assert np.array_equal(a[77:677], b)


def test_uniformity():
    u = rng.uniform_fill_f64(20201217, 0, 0, 1 << 18)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    v = rng.uniform_fill_f32(20201217, 1, 0, 1 << 18).astype(np.float64)
    assert stats.kstest(v, "uniform").pvalue > 1e-4
    h = np.histogram(u, bins=64, range=(0, 1))[0]
    assert stats.chisquare(h).pvalue > 1e-4


def test_path_streams_share_hi_word():
    u53, u24 = rng.path_u53_u24(5, np.arange(10), rng.stream_tag(3, 2), 8)
    k = np.floor(u53 * 2.0 ** 23)
    assert np.array_equal(((k + 0.5) * 2.0 ** -23).astype(np.float32), u24)


# ---------------------------------------------------- single-precision form
@pytest.mark.parametrize("T,d", [(8, 1), (16, 1), (32, 1), (8, 3), (16, 3), (32, 3)])
def test_dyadic_transform_f32_against_fp64(T, d):
    # Algorithm 1 in FP32 (dyadic_transform_f32) against the FP64 evaluation
    # of the same FP32-rounded table, on 2^20 inputs that populate every row
    # (a plain + log-uniform-tail mix) plus every Table 1 boundary and its
    # neighbours.  Row indices agree exactly.  Degree 1 is one fused
    # multiply-add: the result is the FP64 value rounded once, so the error is
    # at most half an FP32 ulp.  Degree 3 is Horner's rule with three FMAs:
    # each rounds once, so |z32 - z| <= gamma_3 sum_j |c_j| s^j with
    # gamma_3 = 3u/(1 - 3u), u = 2^-24 (the standard bound for Horner's rule
    # with fused multiply-adds).
    from tests.inputs import edge_uniforms, random_uniforms
    tab = np.asarray(tables.dyadic_table(T, d), np.float64).astype(np.float32).astype(np.float64)
    u = np.concatenate([random_uniforms(1 << 20, 100 + T + d, np.float32), edge_uniforms(np.float32)])
    u = u[~np.isnan(u)]
    z32, e32 = transform.dyadic_transform_f32(tab, u)
    z64, e64 = transform.dyadic_transform(tab, u.astype(np.float64))
    assert np.array_equal(e32, e64)
    assert set(np.unique(e64)) == set(range(T))  # every row visited
    err = np.abs(z32.astype(np.float64) - z64)
    if d == 1:
        half_ulp = 0.5 * np.spacing(np.abs(z64).astype(np.float32)).astype(np.float64)
        assert np.all(err <= half_ulp * (1.0 + 2.0 ** -28))
    else:
        _, p, ur = transform.dyadic_index(T, u.astype(np.float64))
        s = np.ldexp(ur, e64 + 1)
        absval = sum(np.abs(tab[e64, j]) * s ** j for j in range(d + 1))
        g3 = 3 * 2.0 ** -24 / (1 - 3 * 2.0 ** -24)
        assert np.all(err <= g3 * absval)
        assert err.max() > 0.0  # the FP32 path does round
    # sign handling: z(1 - u) = -z(u) bit for bit where 1 - u is exact in FP32
    v = (np.float32(1.0) - u.astype(np.float32))
    ok = (np.float32(1.0) - v) == u.astype(np.float32)
    zv, _ = transform.dyadic_transform_f32(tab, v[ok])
    assert np.array_equal(zv, -z32[ok])
