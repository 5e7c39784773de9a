"""Gaussian CDF, density and inverse CDF in FP64 (oracle; test infrastructure).

Section 2 of the paper names Phi, phi and Phi^-1 (the exact inverse CDF used by
the inverse transform method).  The paper does not fix an exact routine, so the
oracle takes the plain definition: Phi(z) = erfc(-z/sqrt(2))/2 and Phi^-1(u) is
the root of Phi(z) = u, found by bisection on the lower half u <= 1/2 until the
bracket is two adjacent doubles, then reflected by antisymmetry.
"""
import math

import numpy as np
from scipy.special import erf, erfc

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)

# Phi(-Z_FLOOR) underflows to zero in FP64, so the root of Phi(z) = u for any
# positive double u lies above -Z_FLOOR.
Z_FLOOR = 40.0


def Phi(z):
    """Standard normal CDF, Phi(z) = erfc(-z/sqrt 2)/2 (Section 2 notation)."""
    return 0.5 * erfc(-np.asarray(z, dtype=np.float64) / SQRT2)


def phi(z):
    """Standard normal density; phi(+-inf) = 0 (Section 2 notation)."""
    z = np.asarray(z, dtype=np.float64)
    with np.errstate(over="ignore"):
        return INV_SQRT_2PI * np.exp(-0.5 * z * z)


def _residual(z, q):
    """Phi(z) - q, evaluated through erf when q >= 1/4 (see Phi_inv)."""
    central = q >= 0.25
    r_central = 0.5 * erf(z / SQRT2) - (q - 0.5)
    r_tail = Phi(z) - q
    return np.where(central, r_central, r_tail)


def Phi_inv(u):
    """Exact inverse normal CDF Phi^-1(u) in FP64 (Section 2, Section 3.1).

    For q = min(u, 1-u) (1-u is exact for u >= 1/2) the root z <= 0 of
    Phi(z) = q is bracketed in [-40, 0] and bisected until the bracket holds
    two adjacent doubles; the end with the smaller residual is returned and
    the sign restored (Phi^-1(1-u) = -Phi^-1(u)).  u = 0 and u = 1 give -inf
    and +inf, u outside [0, 1] or NaN gives NaN.

    For q >= 1/4 the same equation is written Phi(z) - 1/2 = erf(z/sqrt2)/2
    = q - 1/2 (the subtraction is exact there), so that roots near z = 0
    keep their relative accuracy.
    """
    u = np.asarray(u, dtype=np.float64)
    scalar = u.ndim == 0
    u = np.atleast_1d(u)
    upper = u > 0.5
    q = np.where(upper, 1.0 - u, u)
    valid = (q > 0.0) & (q <= 0.5)
    qv = np.where(valid, q, 0.25)
    lo = np.where(qv == 0.5, 0.0, -Z_FLOOR)
    hi = np.zeros(qv.shape)
    for _ in range(1200):
        mid = 0.5 * (lo + hi)
        active = (mid != lo) & (mid != hi)
        if not active.any():
            break
        below = _residual(mid, qv) < 0.0
        lo = np.where(active & below, mid, lo)
        hi = np.where(active & ~below, mid, hi)
    rlo = np.abs(_residual(lo, qv))
    rhi = np.abs(_residual(hi, qv))
    z = np.where(rlo < rhi, lo, hi)
    z = np.where(qv == 0.5, 0.0, z)
    z = np.where(upper, -z, z)
    z = np.where(q == 0.0, np.where(upper, np.inf, -np.inf), z)
    z = np.where(np.isnan(u) | (u < 0.0) | (u > 1.0), np.nan, z)
    return z[0] if scalar else z
