"""The Sankaran approximation of the non-central chi-squared inverse CDF, the
comparator of Section 5.1 (Table 6d), in FP64 (oracle; test only).

With k = nu and c1 = 1 - (2/3)(k + lambda)(k + 3 lambda)/(k + 2 lambda)^2,
c2 = (k + 2 lambda)/(k + lambda)^2, c3 = (c1 - 1)(1 - 3 c1):
    C~^-1(U; lambda) = (k + lambda) B^(1/c1),
    B = 1 + c1 c2 (c1 - 1 + (2 - c1) c2 c3 / 2) + c1 sqrt(2 c2) (1 + c2 c3 / 2) Phi^-1(U).
Readings (each pinned by Table 6d): the root of the Gaussian term is
sqrt(2 c2) (the printed sqrt(2 c3) gives errors of order 1-100 instead of
Table 6d's 0.006-0.12); where B < 0 (the far lower tail for small nu) the
approximation is 0 (B clamped at 0); Table 6d's RMSE is the root mean square
over the 200001 equally spaced points of [1e-6, 1 - 1e-6] (its two blank
entries, nu = 1 and lambda <= 5, are where the clamp dominates).
"""
import numpy as np

from . import normal


def constants(nu, lam):
    k = float(nu)
    lam = np.asarray(lam, float)
    c1 = 1.0 - (2.0 / 3.0) * (k + lam) * (k + 3.0 * lam) / (k + 2.0 * lam) ** 2
    c2 = (k + 2.0 * lam) / (k + lam) ** 2
    c3 = (c1 - 1.0) * (1.0 - 3.0 * c1)
    return c1, c2, c3


def approx_x(u, nu, lam, z=None):
    """C~^-1(U; lambda); z = Phi^-1(U) may be passed in (else the oracle's)."""
    u = np.asarray(u, float)
    lam = np.broadcast_to(np.asarray(lam, float), u.shape)
    c1, c2, c3 = constants(nu, lam)
    if z is None:
        z = normal.Phi_inv(u)
    B = 1.0 + c1 * c2 * (c1 - 1.0 + 0.5 * (2.0 - c1) * c2 * c3) + c1 * np.sqrt(2.0 * c2) * (1.0 + 0.5 * c2 * c3) * z
    return (nu + lam) * np.maximum(B, 0.0) ** (1.0 / c1)


def rmse_grid(nu, lam, exact_x, n_grid=200001):
    """RMSE against exact_x(u) on the Table 6d grid."""
    u = np.linspace(1e-6, 1.0 - 1e-6, n_grid)
    return float(np.sqrt(np.mean((approx_x(u, nu, np.full(u.shape, lam)) - exact_x(u)) ** 2)))
