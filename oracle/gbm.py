"""Coupled fine/coarse GBM level replay in FP64 (oracle; test infrastructure).

Section 4: dX = a dt + b dW with a = r X, b = sigma X (geometric Brownian
motion, Section 4.1).  Level l uses 2^l fine steps of delta = T / 2^l and, for
l >= 1, 2^(l-1) coarse steps of 2 delta driven by the pairwise sums of the fine
Wiener increments.  Exact normals Z = Phi^-1(U) and approximate normals
Z~ = approximation(U) come from the same uniform U (Section 4.1).

Schemes
  EM        X <- X + r X delta + sigma X dW                    (Section 4)
  Milstein  X <- X + r X delta + sigma X dW
                   + sigma^2 X (dW^2 - delta) / 2
            (the paper names the Milstein scheme without printing it; this
            is the textbook scheme for b = sigma X, b b' = sigma^2 X.  In one
            dimension the coarse step needs no Levy area.)
Payoffs
  0  P = X_T                         (the functional of Section 4.1's figures)
  1  P = exp(-r T) max(X_T - K, 0)   (discounted European call)
Kinds (Section 4, nested estimator of Section 4.1)
  EXACT       Y = P^_f - P^_c                (two-word draws, Z from u53)
  APPROX      Y = P~_f - P~_c                (one-word draws, Z~ from u24)
  CORRECTION  Y = P^_f - P^_c - P~_f + P~_c  (two-word draws; Z from u53,
                                              Z~ from the u24 of the same draw)
with P_{-1} = 0 at level 0.  The three kinds draw from independent streams
(stream kinds 0, 1, 2), which realises the independent sample sets (i, l) and
(i, l + L + 1) of the nested estimator.
"""
import numpy as np

from . import rng
from .normal import Phi_inv
from .tables import geometric_transform
from .transform import const_transform, dyadic_transform, dyadic_transform_f32

EXACT, APPROX, CORRECTION = 0, 1, 2


def approx_normals(table, u):
    """Z~ from a table: ('dyadic', T x (d+1) array) evaluated in FP64,
    ('dyadic_f32', table) evaluated in FP32 as Code 2 does, ('geometric',
    (table, r)) evaluated in FP64 (Theorem 2.5 with decay rate r), or
    ('const', Q)."""
    kind, tab = table
    if kind == "dyadic":
        return dyadic_transform(tab, u)[0]
    if kind == "geometric":
        return geometric_transform(tab[0], tab[1], u)
    if kind == "dyadic_f32":
        return dyadic_transform_f32(tab, u)[0].astype(np.float64)
    return const_transform(tab, u)


def _paths(params, level, Z):
    """Fine and coarse terminal values driven by the (n_paths, 2^l) normals Z."""
    S0, r, sigma, T = params["S0"], params["r"], params["sigma"], params["T"]
    milstein = params.get("scheme", 0) == 1
    nf = 1 << level
    dt = T / nf
    dW = np.sqrt(dt) * Z

    def step(X, dw, h):
        X2 = X + r * X * h + sigma * X * dw
        if milstein:
            X2 = X2 + 0.5 * sigma * sigma * X * (dw * dw - h)
        return X2

    Xf = np.full(Z.shape[0], float(S0))
    for n in range(nf):
        Xf = step(Xf, dW[:, n], dt)
    if level == 0:
        return Xf, None
    Xc = np.full(Z.shape[0], float(S0))
    for n in range(nf // 2):
        Xc = step(Xc, dW[:, 2 * n] + dW[:, 2 * n + 1], 2.0 * dt)
    return Xf, Xc


def _payoff(params, X):
    if X is None:
        return None
    if params.get("payoff", 0) == 1:
        return np.exp(-params["r"] * params["T"]) * np.maximum(X - params["K"], 0.0)
    return X


def level_replay(params, level, kind, seed, paths, table=None):
    """Per-path (Y, P_f, P_c) for the given global path indices.

    P_f, P_c belong to the exact path for EXACT and CORRECTION and to the
    approximate path for APPROX; P_c = 0 at level 0.
    """
    paths = np.asarray(paths, dtype=np.uint64)
    nf = 1 << level
    tag = rng.stream_tag(level, kind)
    if kind == APPROX:
        u = rng.path_u24(seed, paths, tag, nf).astype(np.float64)
        Zt = approx_normals(table, u)
        Xf, Xc = _paths(params, level, Zt)
        Pf, Pc = _payoff(params, Xf), _payoff(params, Xc)
        Pc = np.zeros_like(Pf) if Pc is None else Pc
        return Pf - Pc, Pf, Pc
    u53, u24 = rng.path_u53_u24(seed, paths, tag, nf)
    Z = Phi_inv(u53)
    Xf, Xc = _paths(params, level, Z)
    Pf, Pc = _payoff(params, Xf), _payoff(params, Xc)
    Pc = np.zeros_like(Pf) if Pc is None else Pc
    if kind == EXACT:
        return Pf - Pc, Pf, Pc
    Zt = approx_normals(table, u24.astype(np.float64))
    Xtf, Xtc = _paths(params, level, Zt)
    Ptf, Ptc = _payoff(params, Xtf), _payoff(params, Xtc)
    Ptc = np.zeros_like(Ptf) if Ptc is None else Ptc
    return (Pf - Pc) - (Ptf - Ptc), Pf, Pc


def em_mean(params, level):
    """E(X_N) of the EM scheme: (1 + r delta)^N, for exact or any
    antisymmetric approximate normals (E Z = 0 and independent steps)."""
    N = 1 << level
    return params["S0"] * (1.0 + params["r"] * params["T"] / N) ** N


def milstein_mean(params, level, second_moment=1.0):
    """E(X_N) of the Milstein scheme when E Z = 0 and E Z^2 = m2:
    every step multiplies the mean by 1 + r delta + sigma^2 delta (m2 - 1)/2."""
    N = 1 << level
    dt = params["T"] / N
    g = 1.0 + params["r"] * dt + 0.5 * params["sigma"] ** 2 * dt * (second_moment - 1.0)
    return params["S0"] * g ** N


def black_scholes_call(params):
    """Discounted call price under GBM (the level-to-infinity limit)."""
    from .normal import Phi
    S0, r, s, T, K = (params[k] for k in ("S0", "r", "sigma", "T", "K"))
    d1 = (np.log(S0 / K) + (r + 0.5 * s * s) * T) / (s * np.sqrt(T))
    d2 = d1 - s * np.sqrt(T)
    return float(S0 * Phi(d1) - K * np.exp(-r * T) * Phi(d2))
