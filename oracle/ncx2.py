"""Non-central chi-squared CDF and inverse CDF in FP64 (oracle; test only).

Section 5: chi^2_nu(lambda) with nu > 0 degrees of freedom and non-centrality
lambda >= 0; C_nu(x; lambda) is its CDF and C_nu^-1(.; lambda) the inverse.
The paper computes the exact inverse by root finding on the CDF, the CDF being
the Poisson mixture of central chi-squared CDFs (Abramowitz and Stegun
26.4.25, which the paper cites):
    C_nu(x; lambda) = sum_j e^(-lambda/2) (lambda/2)^j / j!  P(nu/2 + j, x/2)
with P the regularised lower incomplete gamma function (a library primitive
here).  The oracle sums a window of +-(12 sqrt(lambda/2) + 40) terms around
the Poisson mode, far past FP64 resolution.  The complement uses Q = 1 - P
term by term.  The inverse bisects in log x to a relative width of 4e-16.

Section 5.1's rescaled variable:
    P_nu(U; y) with y = nu / (lambda + nu):
    C_nu^-1(U; lambda) = lambda + nu + 2 sqrt(lambda + nu) P,
so P = (x - lambda - nu) / (2 sqrt(lambda + nu)).
"""
import numpy as np
from scipy.special import gammainc, gammaincc, gammaln


def _terms(lam):
    lam = np.asarray(lam, dtype=np.float64)
    half = 0.5 * lam
    j0 = np.floor(half)
    width = np.ceil(12.0 * np.sqrt(half) + 40.0)
    lo = np.maximum(j0 - width, 0.0)
    n = int(np.max(j0 + width - lo)) + 1
    j = lo[..., None] + np.arange(n, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        logw = -half[..., None] + j * np.log(half[..., None]) - gammaln(j + 1.0)
    logw = np.where(half[..., None] == 0.0, np.where(j == 0.0, 0.0, -np.inf), logw)
    return j, np.exp(logw)


def cdf(x, nu, lam):
    """C_nu(x; lambda), elementwise (broadcast of x and lambda)."""
    x, lam = np.broadcast_arrays(np.asarray(x, float), np.asarray(lam, float))
    j, w = _terms(lam)
    P = gammainc(0.5 * nu + j, 0.5 * np.maximum(x, 0.0)[..., None])
    return np.sum(w * P, axis=-1)


def sf(x, nu, lam):
    """1 - C_nu(x; lambda) summed from the complements term by term."""
    x, lam = np.broadcast_arrays(np.asarray(x, float), np.asarray(lam, float))
    j, w = _terms(lam)
    Q = gammaincc(0.5 * nu + j, 0.5 * np.maximum(x, 0.0)[..., None])
    return np.sum(w * Q, axis=-1)


def icdf(u, nu, lam):
    """C_nu^-1(u; lambda) by bisection in log x (Section 5).

    u <= 1/2 solves C = u; u > 1/2 solves 1 - C = 1 - u (exact subtraction),
    so both tails keep relative accuracy.  Returns 0 for u = 0, inf for u = 1.
    """
    u, lam = np.broadcast_arrays(np.asarray(u, float), np.asarray(lam, float))
    u, lam = u.ravel().copy(), lam.ravel().copy()
    upper = u > 0.5
    target = np.where(upper, 1.0 - u, u)

    def g(logx):  # monotone increasing in log x, root where g = 0
        x = np.exp(logx)
        return np.where(upper, target - sf(x, nu, lam), cdf(x, nu, lam) - target)

    lo = np.full(u.shape, np.log(1e-300))
    hi = np.log(lam + nu + 40.0 * np.sqrt(2.0 * (nu + 2.0 * lam)) + 200.0)
    for _ in range(60):  # widen the upper end until it brackets the root
        bad = g(hi) < 0.0
        if not bad.any():
            break
        hi = np.where(bad, hi + np.log(2.0), hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        done = (hi - lo) <= 4e-16 * np.maximum(np.abs(hi), 1.0)
        if done.all():
            break
        pos = g(mid) >= 0.0
        hi = np.where(~done & pos, mid, hi)
        lo = np.where(~done & ~pos, mid, lo)
    x = np.exp(0.5 * (lo + hi))
    x = np.where(u == 0.0, 0.0, x)
    x = np.where(u == 1.0, np.inf, x)
    return x


def P_from_x(x, nu, lam):
    """Section 5.1's rescaled value P = (x - lambda - nu) / (2 sqrt(lambda + nu))."""
    s = np.asarray(lam, float) + nu
    return (np.asarray(x, float) - s) / (2.0 * np.sqrt(s))


def x_from_P(P, nu, lam):
    s = np.asarray(lam, float) + nu
    return s + 2.0 * np.sqrt(s) * np.asarray(P, float)
