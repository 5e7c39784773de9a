"""Pins of the non-central chi-squared oracle (Section 5), the CIR transition
(Section 5.2) and the surrogate network's FP64 forward/backward."""
import numpy as np
import pytest
from scipy import integrate, stats

from oracle import cir, mlp, ncx2
from oracle.normal import Phi, Phi_inv

NU = 4 * 0.5 * 0.04 / 0.3 ** 2
CIR = dict(kappa=0.5, theta=0.04, xi=0.3, v0=0.04, T=1.0, functional=0)


def test_nu1_closed_form_cdf():
    # chi^2_1(lambda) = (Z + sqrt(lambda))^2
    rng = np.random.default_rng(1)
    x = np.exp(rng.uniform(-6, 6, 80))
    lam = np.exp(rng.uniform(-4, 6, 80))
    ref = Phi(np.sqrt(x) - np.sqrt(lam)) - Phi(-np.sqrt(x) - np.sqrt(lam))
    assert np.allclose(ncx2.cdf(x, 1.0, lam), ref, rtol=1e-12, atol=1e-15)


def test_nu2_lambda0_exponential():
    u = np.array([0.3, 1e-8, 0.999999])
    x = ncx2.icdf(u, 2.0, np.zeros(3))
    assert np.allclose(x, -2.0 * np.log1p(-u), rtol=1e-13)


def test_against_scipy_cdflib():
    # scipy's ncx2 (CDFLIB, the library the paper times against)
    rng = np.random.default_rng(2)
    u = np.concatenate([rng.random(60) * 0.5, 10.0 ** rng.uniform(-12, -2, 20)])
    lam = np.exp(rng.uniform(-8, 7.6, 80))
    x = ncx2.icdf(u, NU, lam)
    assert np.allclose(x, stats.ncx2.ppf(u, NU, lam), rtol=1e-10, atol=0)
    # upper tail: CDFLIB's inverse works on the CDF and loses the tail digits,
    # so the pin is its survival function at the oracle's root
    q = np.concatenate([rng.random(30) * 0.5, 10.0 ** rng.uniform(-12, -2, 20)])
    lam = np.exp(rng.uniform(-8, 7.6, 50))
    x = ncx2.icdf(1.0 - q, NU, lam)
    qq = 1.0 - (1.0 - q)  # the tail mass actually requested
    assert np.allclose(stats.ncx2.sf(x, NU, lam), qq, rtol=1e-11, atol=0)


def test_central_limit_lambda_zero():
    u = np.array([0.01, 0.5, 0.9])
    assert np.allclose(ncx2.icdf(u, NU, np.zeros(3)), stats.chi2.ppf(u, NU), rtol=1e-11)


def test_mean_by_quadrature():
    # int_0^inf (1 - C(x)) dx = nu + lambda
    for lam in (0.5, 20.0, 300.0):
        m, _ = integrate.quad(lambda x: float(ncx2.sf(np.array([x]), NU, np.array([lam]))[0]),
                              0, lam + 60 * np.sqrt(NU + 2 * lam) + 200, limit=400)
        assert m == pytest.approx(NU + lam, rel=1e-8)


def test_rescaled_limit_y_to_zero():
    # Section 5.1: P_nu(U; y) -> Phi^-1(U) as y -> 0 (lambda -> infinity)
    u = np.array([0.05, 0.3, 0.7, 0.95])
    errs = []
    for lam in (1e2, 1e3, 1e4):
        P = ncx2.P_from_x(ncx2.icdf(u, NU, np.full(4, lam)), NU, lam)
        errs.append(np.max(np.abs(P - Phi_inv(u))))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-2


def test_rescaled_limit_y_to_one():
    # y -> 1 (lambda -> 0): P -> C^-1_nu(U) / (2 sqrt nu) - sqrt(nu) / 2
    u = np.array([0.1, 0.5, 0.9])
    P = ncx2.P_from_x(ncx2.icdf(u, NU, np.full(3, 1e-12)), NU, 1e-12)
    assert np.allclose(P, stats.chi2.ppf(u, NU) / (2 * np.sqrt(NU)) - np.sqrt(NU) / 2, rtol=1e-9)


def test_cir_transition_constants():
    nu, c, decay, dt = cir.transition_constants(CIR, 0)
    assert nu == pytest.approx(0.888888888888889)
    assert c == pytest.approx(0.0177061, rel=1e-5)
    assert 0.04 * decay / c == pytest.approx(1.37022, rel=1e-5)
    nu, c, decay, dt = cir.transition_constants(CIR, 6)
    assert 0.04 * decay / c == pytest.approx(113.334, rel=1e-5)


def test_cir_conditional_moments_by_quadrature():
    # E(v1 | v0) = v0 e^-kappa dt + theta (1 - e^-kappa dt); Var = 2 c^2 (nu + 2 lambda)
    nu, c, decay, dt = cir.transition_constants(CIR, 2)
    v0 = 0.04
    lam = v0 * decay / c
    m, var = cir.conditional_moments(CIR, 2, v0)
    assert m == pytest.approx(v0 * decay + 0.04 * (1 - decay), rel=1e-14)
    # the same moments from the CDF: E x = int sf, E x^2 = int 2 x sf
    e1 = integrate.quad(lambda x: float(ncx2.sf(np.array([x]), nu, np.array([lam]))[0]), 0, 400, limit=400)[0]
    e2 = integrate.quad(lambda x: 2 * x * float(ncx2.sf(np.array([x]), nu, np.array([lam]))[0]), 0, 400, limit=400)[0]
    assert c * e1 == pytest.approx(m, rel=1e-8)
    assert c * c * (e2 - e1 * e1) == pytest.approx(var, rel=1e-6)


@pytest.mark.slow
def test_cir_level0_mean():
    n = 2000
    p = dict(CIR, functional=0)
    Y, Pf, Pc = cir.level_replay(p, 0, cir.EXACT, 3, np.arange(n))
    assert abs(Pf.mean() - cir.mean_v(p, 1.0)) < 5 * Pf.std() / np.sqrt(n)
    # E v_T = 0.04 and Var v_T = 0.0022756340 for these parameters
    assert abs(Pf.var() - 0.0022756340) < 0.25 * 0.0022756340


def test_cir_coarse_is_even_subsample():
    p = dict(CIR, functional=0)
    Y, Pf, Pc = cir.level_replay(p, 2, cir.EXACT, 4, np.arange(8))
    assert np.all(Y == 0.0)
    t = cir.mean_time_average(dict(CIR, functional=1), 3)
    assert t == pytest.approx(0.04)


def test_time_average_is_trapezoidal():
    # Section 5.2's path-dependent functional on the level's grid, checked on
    # deterministic paths against closed forms of the trapezoidal rule (a
    # plain mean over the 2^l + 1 nodes, or a missing half weight at either
    # end, gives different values on every path below):
    #   v(t) = t^2 on [0, 1]: (1/N) sum'' (n/N)^2 = 1/3 + 1/(6 N^2)
    #   v(t) = e^(-a t):      (1/N) sum'' q^n = (1 - q^N)(1 + q) / (2 N (1 - q)),  q = e^(-a/N)
    # (sum'' halves the end terms); the coarse value is the same rule on the
    # even nodes (N/2 intervals).
    p = dict(CIR, functional=1)
    for level in (1, 2, 3, 5):
        N = 1 << level
        t = np.linspace(0.0, 1.0, N + 1)
        v = np.stack([t * t, np.exp(-0.7 * t), 0.09 + 0.0 * t])
        Pf, Pc = cir.functional_pair(p, level, v)

        def expo(M, a=0.7):
            q = np.exp(-a / M)
            return (1.0 - q ** M) * (1.0 + q) / (2.0 * M * (1.0 - q))

        M = N // 2
        assert Pf[0] == pytest.approx(1.0 / 3.0 + 1.0 / (6.0 * N * N), rel=1e-13)
        assert Pf[1] == pytest.approx(expo(N), rel=1e-13)
        assert Pf[2] == pytest.approx(0.09, rel=1e-14)
        assert Pc[0] == pytest.approx(1.0 / 3.0 + 1.0 / (6.0 * M * M), rel=1e-13)
        assert Pc[1] == pytest.approx(expo(M), rel=1e-13)
    # level 0: one step, P_f = (v_0 + v_1)/2 and no coarse path
    Pf, Pc = cir.functional_pair(p, 0, np.array([[0.09, 0.05]]))
    assert Pf[0] == pytest.approx(0.07) and Pc[0] == 0.0


def test_time_average_closed_form_off_equilibrium():
    # v0 = 0.09 != theta: the mean of the time average is the trapezoidal
    # rule applied to E v_t = theta + (v0 - theta) e^(-kappa t); at level 0
    # (one transition) it is (v0 + E v_T) / 2, and it differs from the plain
    # mean over the nodes at every level >= 1
    p = dict(CIR, functional=1, v0=0.09)
    assert cir.mean_time_average(p, 0) == pytest.approx(0.5 * (0.09 + cir.mean_v(p, 1.0)), rel=1e-15)
    for level in (1, 2, 4):
        t = np.linspace(0.0, 1.0, (1 << level) + 1)
        assert abs(cir.mean_time_average(p, level) - cir.mean_v(p, t).mean()) > 1e-5


# ---------------------------------------------------------------- MLP
def test_mlp_finite_differences():
    p = mlp.init_params(5)
    rng = np.random.default_rng(6)
    w, g, t = rng.normal(size=32), rng.uniform(-1, 1, 32), rng.normal(size=32)
    L, grads = mlp.loss_and_grads(p, w, g, t, bf16=False)
    for name in mlp.PARAM_ORDER:
        flat = np.atleast_1d(p[name]).ravel()
        idxs = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idxs:
            h = 1e-6
            pp = {k: np.array(v, dtype=float, copy=True) for k, v in p.items()}
            pm = {k: np.array(v, dtype=float, copy=True) for k, v in p.items()}
            pp[name].reshape(-1)[i] += h
            pm[name].reshape(-1)[i] -= h
            fd = (mlp.loss_and_grads(pp, w, g, t, bf16=False)[0] - mlp.loss_and_grads(pm, w, g, t, bf16=False)[0]) / (2 * h)
            an = np.atleast_1d(grads[name]).reshape(-1)[i]
            assert fd == pytest.approx(an, rel=1e-6, abs=1e-9)


def test_mlp_hand_case():
    # unit 0 of layer 1 passes w through relu; unit 3 of layer 2 adds it to
    # its bias 2; unit 5 of layer 2 has a negative input (-3) that relu
    # removes, whatever its output weight:
    #   w = 1.5:  h1[0] = 1.5, a2[3] = 3.5, P = 1.5 + 0.5 * 3.5 + 0.25 = 3.5
    #   w = -2:   h1[0] = 0,   a2[3] = 2,   P = -2 + 0.5 * 2 + 0.25 = -0.75
    p = {k: np.zeros(s) for k, s in mlp.PARAM_SHAPES.items()}
    p["W1"][0, 0] = 1.0
    p["W2"][3, 0] = 1.0
    p["b2"][3] = 2.0
    p["W3"][3] = 0.5
    p["b2"][5] = -3.0
    p["W3"][5] = 7.0
    p["b3"] = np.array(0.25)
    P = mlp.forward(p, np.array([1.5, -2.0]), np.array([0.0, 0.3]))
    assert np.array_equal(P, np.array([3.5, -0.75]))


def test_truncated_em_step_closed_form():
    # v' = v + kappa (theta - v) delta + xi sqrt(|v| delta) Phi^-1(u): at u = 1/2
    # the drift alone; antisymmetric in Phi^-1(u) about it; |v| under the root
    from oracle import normal
    p = dict(v0=1.0, kappa=0.5, theta=1.0, xi=1.0, T=1.0, functional=0)
    level = 3
    nu, c, decay, dt = cir.transition_constants(p, level)
    f = cir.em_x(p, level)
    for v in (2.0, 0.3, -0.05):
        lam = np.array([v * decay / c])
        drift = v + 0.5 * (1.0 - v) * dt
        assert np.isclose(f(np.array([0.5]), lam)[0] * c, drift, rtol=0, atol=1e-15)
        for u in (0.01, 0.3):
            up = f(np.array([1 - u]), lam)[0] * c
            lo = f(np.array([u]), lam)[0] * c
            assert np.isclose(0.5 * (up + lo), drift, rtol=0, atol=1e-14)
            z = normal.Phi_inv(np.array([1 - u]))[0]
            assert np.isclose(up - drift, np.sqrt(abs(v) * dt) * z, rtol=1e-13)


def test_twoway_replay_is_fine_difference():
    # TWOWAY returns P^_f - P~_f on the CORRECTION draws, with (P^_f, P~_f)
    p = dict(CIR, functional=1)
    em = cir.em_x(p, 2)
    Y, Pf, Pt = cir.level_replay(p, 2, cir.TWOWAY, 5, np.arange(6), surrogate_x=em)
    assert np.allclose(Y, Pf - Pt, rtol=0, atol=0)
    Yc, Pfc, _ = cir.level_replay(p, 2, cir.CORRECTION, 5, np.arange(6), surrogate_x=em)
    assert not np.allclose(Pf, Pfc)  # another stream (kind 7 vs 6)


def test_mlp_split_layer1():
    # the split-BF16 layer 1 of the inference kernels: exact when every
    # value is a BF16 number, and within ~2^-16 relative of the exact a1
    # otherwise (the dropped lo x lo products and the second-level residues)
    rng = np.random.default_rng(11)
    p = mlp.init_params(3)
    p = {k: np.asarray(v, float).astype(np.float32).astype(np.float64) for k, v in p.items()}
    w = rng.normal(size=500).astype(np.float32).astype(np.float64)
    g = rng.uniform(-1, 1, 500).astype(np.float32).astype(np.float64)
    exact = np.stack([w, g], axis=-1) @ p["W1"].T + p["b1"]
    split = mlp.layer1_split(p, w, g)
    scale = np.abs(w)[:, None] * np.abs(p["W1"][:, 0]) + np.abs(g)[:, None] * np.abs(p["W1"][:, 1]) + np.abs(p["b1"])
    assert np.all(np.abs(split - exact) <= 2.0 ** -15 * scale)
    assert np.any(split != exact)
    from oracle.dtypes import round_bf16
    q = {k: round_bf16(v) for k, v in p.items()}
    wq, gq = round_bf16(w), round_bf16(g)
    assert np.array_equal(mlp.layer1_split(q, wq, gq), np.stack([wq, gq], axis=-1) @ q["W1"].T + q["b1"])
