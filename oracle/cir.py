"""CIR transitions and level replay in FP64 (oracle; test infrastructure).

Section 5.2: dv = kappa (theta - v) dt + xi sqrt(v) dW.  Over a horizon T the
distribution of v_T given v_0 is a scaled non-central chi-squared with
nu = 4 kappa theta / xi^2 and lambda = 4 kappa v_0 e^(-kappa T) /
(xi^2 (1 - e^(-kappa T))).  The paper prints this for the horizon only; the
reading used for one step of size delta is the same result with T -> delta
and v_0 -> v_n (the Markov property):
    c = xi^2 (1 - e^(-kappa delta)) / (4 kappa)
    lambda_n = v_n e^(-kappa delta) / c
    v_(n+1) = c * C_nu^-1(U_n; lambda_n).

Levels.  Level l uses 2^l exact-in-law transitions.  The coarse path of level
l is the fine path observed at even steps, which has the law of the 2^(l-1)
step chain, so the coupling is exact.  Functionals
  0  P = v_T      (then P_l - P_(l-1) = 0 for l >= 1)
  1  P = the trapezoidal time average of the path on the level's grid
     (the arithmetic average of Section 5.2's path-dependent example).
Kinds: EXACT (stream kind 4, u53 draws, exact inverse), SURROGATE (stream
kind 5, u24 draws, the approximation), CORRECTION (stream kind 6, two-word
draws: exact from u53 and approximation from the u24 of the same draw);
Y = P_f - P_c for the first two and D = (P^_f - P^_c) - (P~_f - P~_c) for the
third; TWOWAY (stream kind 7, the draws of CORRECTION, fine paths only):
Y = P^_f - P~_f, the two-way difference at one time step of Figure 4b.

Truncated Euler-Maruyama (Section 5.2, after Higham and Mao): the Gaussian
scheme the chi-squared approximations are compared with,
    v_(n+1) = v_n + kappa (theta - v_n) delta + xi sqrt(|v_n| delta) Z_n,
with Z_n = Phi^-1(U_n) on the same uniforms.
"""
import numpy as np

from . import ncx2, normal, rng

EXACT, SURROGATE, CORRECTION, TWOWAY = 0, 1, 2, 3
STREAM_BASE = 4


def transition_constants(params, level):
    k, th, xi, T = params["kappa"], params["theta"], params["xi"], params["T"]
    n = 1 << level
    dt = T / n
    nu = 4.0 * k * th / xi ** 2
    c = xi ** 2 * (1.0 - np.exp(-k * dt)) / (4.0 * k)
    decay = np.exp(-k * dt)
    return nu, c, decay, dt


def run_path(params, level, x_of_u_lam, U):
    """Chain v_0..v_N from uniforms U (n_paths, N) through x = x_of_u_lam(u, lam)."""
    nu, c, decay, dt = transition_constants(params, level)
    N = 1 << level
    v = np.empty((U.shape[0], N + 1))
    v[:, 0] = params["v0"]
    for n in range(N):
        lam = v[:, n] * decay / c
        v[:, n + 1] = c * x_of_u_lam(U[:, n], lam)
    return v


def functional_pair(params, level, v):
    """(P_f, P_c) of one path array v (n_paths, 2^l + 1)."""
    N = 1 << level
    if params.get("functional", 0) == 0:
        Pf = v[:, -1]
        Pc = v[:, -1] if level > 0 else np.zeros_like(Pf)
        return Pf, Pc
    Pf = (0.5 * v[:, 0] + v[:, 1:N].sum(axis=1) + 0.5 * v[:, N]) / N
    if level == 0:
        return Pf, np.zeros_like(Pf)
    ve = v[:, ::2]
    M = N // 2
    Pc = (0.5 * ve[:, 0] + ve[:, 1:M].sum(axis=1) + 0.5 * ve[:, M]) / M
    return Pf, Pc


def exact_x(params):
    nu = 4.0 * params["kappa"] * params["theta"] / params["xi"] ** 2
    return lambda u, lam: ncx2.icdf(u, nu, lam)


def em_x(params, level):
    """The truncated Euler-Maruyama step written as x(u, lambda) for run_path:
    v_n = lambda c / e^(-kappa delta), v_(n+1) as above, x = v_(n+1) / c."""
    nu, c, decay, dt = transition_constants(params, level)
    k, th, xi = params["kappa"], params["theta"], params["xi"]

    def f(u, lam):
        v = np.asarray(lam, float) * c / decay
        z = normal.Phi_inv(np.asarray(u, float))
        return (v + k * (th - v) * dt + xi * np.sqrt(np.abs(v) * dt) * z) / c
    return f


def level_replay(params, level, kind, seed, paths, surrogate_x=None):
    """Per-path (Y, P_f, P_c); P_f, P_c of the exact path for EXACT and
    CORRECTION, of the surrogate path for SURROGATE.

    surrogate_x(u, lam) -> x~ implements the surrogate transition (including
    its own fallback rule) on FP64 arrays.
    """
    paths = np.asarray(paths, dtype=np.uint64)
    N = 1 << level
    tag = rng.stream_tag(level, STREAM_BASE + kind)
    if kind == SURROGATE:
        u = rng.path_u24(seed, paths, tag, N).astype(np.float64)
        v = run_path(params, level, surrogate_x, u)
        Pf, Pc = functional_pair(params, level, v)
        return Pf - Pc, Pf, Pc
    u53, u24 = rng.path_u53_u24(seed, paths, tag, N)
    v = run_path(params, level, exact_x(params), u53)
    Pf, Pc = functional_pair(params, level, v)
    if kind == EXACT:
        return Pf - Pc, Pf, Pc
    vt = run_path(params, level, surrogate_x, u24.astype(np.float64))
    Ptf, Ptc = functional_pair(params, level, vt)
    if kind == TWOWAY:
        return Pf - Ptf, Pf, Ptf
    return (Pf - Pc) - (Ptf - Ptc), Pf, Pc


def conditional_moments(params, level, v):
    """E(v_(n+1) | v_n) and Var(v_(n+1) | v_n) of one transition:
    c (nu + lambda) and 2 c^2 (nu + 2 lambda)."""
    nu, c, decay, dt = transition_constants(params, level)
    lam = np.asarray(v, float) * decay / c
    return c * (nu + lam), 2.0 * c * c * (nu + 2.0 * lam)


def mean_v(params, t):
    """E(v_t) = theta + (v_0 - theta) e^(-kappa t)."""
    return params["theta"] + (params["v0"] - params["theta"]) * np.exp(-params["kappa"] * t)


def mean_time_average(params, level):
    """E of the trapezoidal time average on 2^l steps (linear in E v_t)."""
    N = 1 << level
    t = np.linspace(0.0, params["T"], N + 1)
    m = mean_v(params, t)
    return float((0.5 * m[0] + m[1:N].sum() + 0.5 * m[N]) / N)
