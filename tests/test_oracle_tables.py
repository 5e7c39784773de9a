"""Pins of the coefficient tables (Sections 2.2, 2.3, 3.2, 3.3)."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import tables
from oracle.normal import Phi_inv, phi
from tests.conftest import read_golden


def trunc(x, digits):
    """Truncate toward zero to `digits` significant digits."""
    if x == 0:
        return 0.0
    e = math.floor(math.log10(abs(x))) - digits + 1
    return math.trunc(x / 10.0 ** e) * 10.0 ** e


# ---------------------------------------------------------------- constant
def test_code1_printed_values():
    Q = tables.const_table(1024, "E")
    for idx, val in read_golden("code1_const_table.txt"):
        q = float(np.float32(Q[int(idx)]))
        assert math.trunc(q * 10) / 10 == pytest.approx(float(val), abs=1e-12)


@pytest.mark.parametrize("N", [2, 4, 8])
def test_const_conditional_mean_brute_force(N):
    # E(Z | Phi(Z) in I_k) = N * int_{I_k} Phi^-1(u) du, by mpmath quadrature in u
    mp.mp.dps = 30
    Q = tables.const_table(N, "E")
    inv = lambda u: mp.sqrt(2) * mp.erfinv(2 * u - 1)
    for k in range(N):
        ref = N * mp.quad(inv, [mp.mpf(k) / N, mp.mpf(k + 1) / N])
        assert abs(Q[k] - float(ref)) < 1e-12


@pytest.mark.parametrize("construction", ["E", "C", "I"])
def test_const_theorem_2_3_conditions(construction):
    # Theorem 2.3 conditions (symmetry, intermediate values, end growth) and
    # Corollary 2.4's bound Q_K <= z_K + 1.25 q^-1/2 for q >= 10.
    q = 10
    N = 2 ** q
    Q = tables.const_table(N, construction)
    K = N - 1
    assert np.allclose(Q, -Q[::-1], rtol=0, atol=1e-13)
    z = Phi_inv(np.arange(N + 1) / N)
    inner = np.arange(1, K)
    assert np.all(z[inner] <= Q[inner] + 1e-13) and np.all(Q[inner] <= z[inner + 1] + 1e-13)
    assert z[K] <= Q[K] + 1e-13 and Q[K] <= z[K] + 1.25 / math.sqrt(q)


def test_corollary_2_4_end_interval():
    # Q_K - z_K < 9/(8 z_K) for q >= 10 (proof of Corollary 2.4)
    for q in (10, 12, 14):
        N = 2 ** q
        Q = tables.const_table(N)
        zK = float(Phi_inv(1.0 - 1.0 / N))
        assert Q[-1] - zK < 9.0 / (8.0 * zK)


def test_const_rmse_decreases_and_matches_prose():
    Ns = [2, 8, 16, 64, 256, 1024, 4096]
    e = [tables.const_l2_error(tables.const_table(N)) for N in Ns]
    assert all(a > b for a, b in zip(e, e[1:]))
    # Section 2.2: about 1e-2 at ~1000 intervals, a drop of ~10^2 from 2 to 10^3
    assert 0.5e-2 < e[5] < 2e-2
    assert 30 < e[0] / e[5] < 300


@pytest.mark.parametrize("N", [2, 8, 64])
def test_const_projection_identity_vs_quadrature(N):
    Q = tables.const_table(N)
    assert tables.const_l2_error(Q) == pytest.approx(tables.const_lp_error_quad(Q, 2), rel=1e-8)


def test_const_lp_error_falls_with_q():
    # Theorem 2.3 for p = 4: ||Q - Phi^-1||_4^4 = O(2^-q q^-2) -> falls with q
    e = [tables.const_lp_error_quad(tables.const_table(2 ** q), 4) for q in (3, 5, 7)]
    assert e[0] > e[1] > e[2]


# ---------------------------------------------------------------- dyadic
def test_code2_printed_coefficients():
    tab = tables.dyadic_table(16, 1)
    for idx, c0, c1 in read_golden("code2_linear_table.txt"):
        e = int(idx)
        a = tables.to_u_monomials(tab[e], e) if e > 0 else np.zeros(2)
        a32 = a.astype(np.float32).astype(np.float64)
        assert trunc(a32[0], 2) == pytest.approx(float(c0), rel=1e-9, abs=1e-12)
        assert trunc(a32[1], 2) == pytest.approx(float(c1), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("T", [8, 16, 32])
def test_singular_interval_closed_form(T):
    tab = tables.dyadic_table(T, 1)
    e = T - 1
    a = tables.to_u_monomials(tab[e], e)
    alpha, beta = tables.singular_closed_form(2.0 ** -(T - 1))
    assert a[0] == pytest.approx(alpha, rel=1e-10)
    assert a[1] == pytest.approx(beta, rel=1e-10)


def test_degree1_moments_closed_form():
    # int_a^b Phi^-1 = phi(z_a) - phi(z_b); int_a^b u Phi^-1 =
    # a phi(z_a) - b phi(z_b) + (Phi(sqrt2 z_b) - Phi(sqrt2 z_a)) / (2 sqrt(pi))
    from oracle.normal import Phi
    for e in (1, 4, 9):
        a, b, h = tables.dyadic_interval(e, 16)
        za, zb = float(Phi_inv(a)), float(Phi_inv(b))
        I0 = float(phi(za) - phi(zb))
        I1 = a * float(phi(za)) - b * float(phi(zb)) + float(Phi(math.sqrt(2) * zb) - Phi(math.sqrt(2) * za)) / (2 * math.sqrt(math.pi))
        assert tables._moment(0, a, b, h) == pytest.approx(I0, rel=1e-11)
        assert tables._moment(1, a, b, h) * h == pytest.approx(I1, rel=1e-11)


def test_dyadic_brute_force_mpmath_T4():
    # L2 fit on every interval by mpmath quadrature directly in u
    mp.mp.dps = 30
    inv = lambda u: mp.sqrt(2) * mp.erfinv(2 * u - 1)
    for d in (1, 3):
        tab = tables.dyadic_table(4, d)
        for e in range(1, 4):
            a, b, h = tables.dyadic_interval(e, 4)
            G = mp.matrix(d + 1, d + 1)
            m = mp.matrix(d + 1, 1)
            for i in range(d + 1):
                for j in range(d + 1):
                    G[i, j] = mp.quad(lambda u: (u / h) ** (i + j), [a, b])
                m[i] = mp.quad(lambda u: (u / h) ** i * inv(u), [a, b])
            c = mp.lu_solve(G, m)
            for j in range(d + 1):
                assert tab[e, j] == pytest.approx(float(c[j]), rel=1e-9, abs=1e-11)


@pytest.mark.parametrize("T,d", [(8, 1), (16, 1), (16, 3), (32, 3)])
def test_dyadic_residual_orthogonal(T, d):
    # L2 projection: the residual is orthogonal to 1, s, .., s^d on each interval
    from scipy import integrate
    tab = tables.dyadic_table(T, d)
    for e in (1, T // 2, T - 2):
        a, b, h = tables.dyadic_interval(e, T)
        for j in range(d + 1):
            f = lambda u: (u / h) ** j * (float(Phi_inv(u)) - np.polyval(tab[e][::-1], u / h))
            val, _ = integrate.quad(f, a, b, epsabs=1e-16, epsrel=1e-10, limit=200)
            scale = integrate.quad(lambda u: abs((u / h) ** j * float(Phi_inv(u))), a, b)[0]
            assert abs(val) < 1e-9 * scale


@pytest.mark.parametrize("e", [1, 3, 6, 10, 14])
def test_peano_pointwise_bound(e):
    # |eps(u)| <= -6 (b-a)^2 (Phi^-1)''(a) <= 2.59 ((1-r)/r)^2 on non-singular
    # intervals (proof of Theorem 2.5), r = 1/2
    tab = tables.dyadic_table(16, 1)
    a, b, h = tables.dyadic_interval(e, 16)
    za = float(Phi_inv(a))
    d2 = za / float(phi(za)) ** 2  # (Phi^-1)''(u) = z / phi(z)^2
    bound = -6.0 * (b - a) ** 2 * d2
    assert bound <= 2.59
    u = np.linspace(a, b, 2001)[:-1]
    err = np.abs(Phi_inv(u) - np.polyval(tab[e][::-1], u / h))
    assert err.max() <= bound


def test_dyadic_rmse_falls_and_matches_prose():
    r = {(T, d): tables.dyadic_l2_error(tables.dyadic_table(T, d)) for T in (8, 16, 32) for d in (1, 3)}
    for d in (1, 3):
        assert r[(8, d)] > r[(16, d)] > r[(32, d)]
    for T in (8, 16, 32):
        assert r[(T, 3)] < r[(T, 1)]
    # Section 2.3: linear about 1e-2 at 16 intervals, cubic about 1e-4, a drop of ~10^2
    assert 3e-3 < r[(16, 1)] < 2e-2
    assert 1e-4 < r[(16, 3)] < 1e-3
    assert r[(16, 1)] / r[(16, 3)] > 10


@pytest.mark.parametrize("T,d", [(8, 1), (16, 3)])
def test_dyadic_projection_identity_vs_quadrature(T, d):
    tab = tables.dyadic_table(T, d)
    assert tables.dyadic_l2_error(tab) == pytest.approx(tables.dyadic_l2_error_quad(tab), rel=1e-6)


def test_dyadic_zero_entry_and_local_basis_range():
    for T in (8, 16, 32):
        for d in (1, 3):
            tab = tables.dyadic_table(T, d)
            assert np.all(tab[0] == 0.0)
            assert np.abs(tab).max() < 8.0  # fits FP16 (unlike u-monomials)


# ---------------------------------------------------------------- geometric (Theorem 2.5, general r)
@pytest.mark.parametrize("T,d", [(8, 1), (16, 1), (16, 3), (32, 2)])
def test_geometric_half_rate_is_the_dyadic_table(T, d):
    # r = 1/2: the thresholds are the exact powers 2^-(e+1) and s = t 2^(e+1)
    tab = tables.geometric_table(0.5, T, d)
    # the dyadic fit solves the monomial normal equations, which lose ~1e-10
    # for cubics; the geometric fit projects in the Legendre basis
    assert np.allclose(tab, tables.dyadic_table(T, d), rtol=1e-9, atol=1e-9)
    assert np.array_equal(tables.geometric_thresholds(0.5, T), 2.0 ** -(np.arange(T) + 1.0))


@pytest.mark.parametrize("r", [0.3, 0.6, 0.75, 0.9])
def test_geometric_row_is_the_logarithm(r):
    # t in [B_e, B_(e-1)) <=> e = ceil(log(2t) / log r), away from the FP32
    # rounding of the thresholds; the last row also takes everything below
    T = 24
    rng = np.random.default_rng(5)
    t = 0.5 * r ** rng.uniform(0.0, T + 6.0, 20000)
    e_log = np.ceil(np.log(2 * t) / math.log(r))
    frac = e_log - np.log(2 * t) / math.log(r)
    keep = (frac > 1e-5) & (frac < 1 - 1e-5)
    want = np.minimum(e_log, T - 1)
    got = tables.geometric_row(t, r, T)
    assert keep.sum() > 19000
    assert np.array_equal(got[keep], want[keep])
    # boundaries: B_e is in row e, the float below it in row e + 1
    B = tables.geometric_thresholds(r, T)
    for e in range(1, T - 1):
        assert tables.geometric_row(B[e], r, T) == e
        assert tables.geometric_row(np.nextafter(B[e], 0.0), r, T) == e + 1
    assert tables.geometric_row(0.5, r, T) == 0 and tables.geometric_row(0.0, r, T) == T - 1


@pytest.mark.parametrize("r,T", [(0.6, 12), (0.8, 24), (0.9, 40)])
def test_geometric_singular_interval_closed_form(r, T):
    # proof of Theorem 2.5: on (0, b) the linear fit is alpha + beta u with
    # alpha, beta in closed form from z_b = Phi^-1(b); here s = u / B_(T-1)
    tab = tables.geometric_table(r, T, 1)
    a, b, h = tables.geometric_interval(T - 1, r, T)
    assert a == 0.0
    alpha, beta = tables.singular_closed_form(b)
    assert tab[T - 1, 0] == pytest.approx(alpha, rel=1e-10)
    assert tab[T - 1, 1] / h == pytest.approx(beta, rel=1e-10)


@pytest.mark.parametrize("r", [0.6, 0.8, 0.9])
def test_geometric_brute_force_mpmath(r):
    # L2 fit by mpmath quadrature directly in u on a non-singular and the singular row
    mp.mp.dps = 30
    inv = lambda u: mp.sqrt(2) * mp.erfinv(2 * u - 1)
    T, d = 10, 2
    tab = tables.geometric_table(r, T, d)
    for e in (1, 5, T - 1):
        a, b, h = tables.geometric_interval(e, r, T)
        G = mp.matrix(d + 1, d + 1)
        m = mp.matrix(d + 1, 1)
        for i in range(d + 1):
            for j in range(d + 1):
                G[i, j] = mp.quad(lambda u: (u / h) ** (i + j), [a, b])
            m[i] = mp.quad(lambda u: (u / h) ** i * inv(u), [a, b])
        c = mp.lu_solve(G, m)
        # values, not monomial coefficients: for r near 1 the basis 1, s, s^2
        # on [1, 1/r) is nearly collinear and the coefficients ill-conditioned
        s = np.linspace(a / h, b / h, 41)
        want = np.array([float(sum(c[j] * mp.mpf(x) ** j for j in range(d + 1))) for x in s])
        assert np.allclose(np.polyval(tab[e][::-1], s), want, rtol=0, atol=1e-11)


@pytest.mark.parametrize("r", [0.6, 0.75, 0.9])
def test_geometric_peano_pointwise_bound(r):
    # |eps(u)| <= -6 (b-a)^2 (Phi^-1)''(a) <= 2.59 ((1-r)/r)^2 (proof of Theorem 2.5)
    T = 30
    tab = tables.geometric_table(r, T, 1)
    for e in (1, 2, 5, 12, T - 2):
        a, b, h = tables.geometric_interval(e, r, T)
        za = float(Phi_inv(a))
        bound = -6.0 * (b - a) ** 2 * za / float(phi(za)) ** 2
        assert bound <= 2.59 * ((1 - r) / r) ** 2 * (1 + 1e-6)
        u = np.linspace(a, b, 2001)[:-1]
        err = np.abs(Phi_inv(u) - np.polyval(tab[e][::-1], u / h))
        assert err.max() <= bound


@pytest.mark.parametrize("r,T,d", [(0.7, 12, 1), (0.85, 20, 3)])
def test_geometric_projection_identity_vs_quadrature(r, T, d):
    # the RMSE from the projection identity against direct quadrature of
    # (D - Phi^-1)^2 over both halves
    from scipy import integrate
    tab = tables.geometric_table(r, T, d)
    tot = 0.0
    for e in range(1, T):
        a, b, h = tables.geometric_interval(e, r, T)
        f = lambda u: (np.polyval(tab[e][::-1], u / h) - float(Phi_inv(u))) ** 2
        pts = [b * 1e-8, b * 1e-4, b * 1e-2] if a == 0.0 else None
        tot += integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-11, limit=400, points=pts)[0]
    assert tables.geometric_l2_error(tab, r) == pytest.approx(math.sqrt(2 * tot), rel=1e-5)


def test_geometric_theorem_2_5_central_rate():
    # with the singular row negligible (r^(T-1) ~ 1e-30) the error is the
    # central O((1-r)^2) in L2: local log-log slope in (1 - r) near 2 for
    # linear rows, and the cubic rows fall faster
    def rmse(r, d):
        T = int(math.ceil(math.log(1e-30) / math.log(r))) + 1
        return tables.geometric_l2_error(tables.geometric_table(r, T, d), r)

    for d, lo, hi in ((1, 1.8, 2.4), (3, 3.5, 5.5)):
        e8, e9 = rmse(0.8, d), rmse(0.9, d)
        slope = math.log(e8 / e9) / math.log(2.0)
        assert lo < slope < hi, (d, slope)
    assert rmse(0.6, 1) < rmse(0.5, 1) and rmse(0.9, 1) < rmse(0.8, 1)


def test_geometric_theorem_2_5_decoupling():
    # adding intervals at fixed r only shrinks the singular term: the error
    # plateaus at the central one; the singular row's own contribution is of
    # order b / |z_b|^2 with b = r^(T-1)/2
    from scipy import integrate
    for r, Ts in ((0.5, (40, 60, 90)), (0.8, (100, 150, 200))):
        e = [tables.geometric_l2_error(tables.geometric_table(r, T, 1), r) for T in Ts]
        assert abs(e[1] / e[0] - 1) < 0.02 and abs(e[2] / e[1] - 1) < 1e-3
    for r in (0.5, 0.8):
        for T in (8, 16, 24, 32):
            tab = tables.geometric_table(r, T, 1)
            a, b, h = tables.geometric_interval(T - 1, r, T)
            f = lambda u: (np.polyval(tab[T - 1][::-1], u / h) - float(Phi_inv(u))) ** 2
            part = 2 * integrate.quad(f, 0.0, b, epsabs=0.0, epsrel=1e-10, limit=400,
                                      points=[b * 1e-8, b * 1e-4])[0]
            zb = float(Phi_inv(b))
            assert 0.05 < part / (b / zb ** 2) < 1.0, (r, T, part / (b / zb ** 2))


def test_geometric_transform_matches_rows():
    # evaluation: reflection, row choice and local variable against a direct
    # per-sample polynomial evaluation
    r, T, d = 0.7, 20, 3
    tab = tables.geometric_table(r, T, d)
    rng = np.random.default_rng(9)
    u = np.concatenate([rng.random(5000), [0.5, 1e-30, 1 - 1e-12]])
    z = tables.geometric_transform(tab, r, u)
    for k in rng.integers(0, u.size, 300).tolist() + [u.size - 3, u.size - 2, u.size - 1]:
        t = min(u[k], 1 - u[k])
        e = int(tables.geometric_row(np.float64(t), r, T))
        if e == 0:
            want = 0.0
        else:
            h = tables.geometric_interval(e, r, T)[2]
            want = np.polyval(tab[e][::-1], t / h)
        assert z[k] == pytest.approx(want if u[k] < 0.5 else -want, rel=1e-14, abs=1e-14)
    # Phi^-1 increases: the fit may step back only at a row boundary, and by little
    zs = z[np.argsort(u)]
    assert np.all(np.diff(zs) > -0.05)
