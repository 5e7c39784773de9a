"""Applying a coefficient table to uniforms (oracle; test infrastructure).

Piecewise constant, Section 3.2 and Code 1: the interval of u is m = floor(N u)
on [m/N, (m+1)/N).  The paper's loop has no guard for u = 1; the reading here
clamps m to [0, N-1] (so u = 1 uses the last interval), and NaN maps to
interval 0.

Dyadic piecewise polynomial, Algorithm 1 of Section 3.3:
  predicate p = (u < 1/2)       [Algorithm 1 writes U > 1/2 and Code 2 u < 0.5;
                                  both send u = 1/2 to entry 0]
  reflect   u' = u if p else 1 - u     (exact for u >= 1/2)
  index     e = the dyadic interval of u' (Table 1), capped at T - 1
  evaluate  the polynomial of entry e, then negate unless p.
The oracle finds e with frexp (u' = f 2^x, f in [1/2, 1) gives e = -x), not by
reading exponent bits, so it is independent of the bit-level method; u' = 0
(from u = 0 or u = 1) goes to the capped entry.  The polynomial is evaluated
in FP64 in the local variable s = u' 2^(e+1) on the stored (dtype-rounded)
coefficients.
"""
import numpy as np


def const_index(n_intervals, u):
    u = np.asarray(u, dtype=np.float64)
    N = int(n_intervals)
    x = np.where(np.isnan(u), 0.0, u) * N  # exact: N is a power of two
    m = np.floor(np.clip(x, 0.0, float(N - 1)))
    return m.astype(np.int64)


def const_transform(Q, u):
    """z = Q[m(u)] (Code 1, with the clamp described in the module header)."""
    Q = np.asarray(Q, dtype=np.float64)
    return Q[const_index(len(Q), u)]


def dyadic_index(n_entries, u):
    """(e, p, u'): table entry, predicate and reflected input (Algorithm 1)."""
    u = np.asarray(u, dtype=np.float64)
    T = int(n_entries)
    p = u < 0.5
    ur = np.where(p, u, 1.0 - u)
    _, x = np.frexp(ur)
    e = np.minimum(-x, T - 1)
    e = np.where(ur == 0.0, T - 1, e)
    e = np.where(np.isnan(ur), T - 1, e)
    return e.astype(np.int64), p, ur


def dyadic_transform(tab, u):
    """Approximate Phi^-1(u) from a T x (d+1) table in the local variable s.

    Returns (z, e): the FP64 value (sign restored) and the entry index.
    Horner's rule in FP64; for NaN input the value is NaN.
    """
    tab = np.asarray(tab, dtype=np.float64)
    T, d1 = tab.shape
    e, p, ur = dyadic_index(T, u)
    s = np.ldexp(ur, e + 1)
    c = tab[e]
    z = np.zeros(s.shape)
    for j in range(d1 - 1, -1, -1):
        z = z * s + c[..., j]
    z = np.where(p, z, -z)
    return z, e


def fma_f32(a, b, c):
    """Single-precision fused multiply-add: the product of two FP32 values is
    exact in FP64, so one FP64 add and one rounding to FP32 give fma(a, b, c)
    except in the rare double-rounding case (the FP64 sum landing exactly
    half-way between two FP32 values)."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    return (a * b + c).astype(np.float32)


def dyadic_transform_f32(tab, u):
    """Algorithm 1 carried out in single precision, as the paper's Code 2 does:
    FP32 input, FP32 reflection (exact), s = u' 2^(e+1) (exact), Horner's rule
    with FP32 fused multiply-adds over the (FP32) coefficients.  Returns
    (z as float32, e)."""
    tab = np.asarray(tab, dtype=np.float64).astype(np.float32)
    u32 = np.asarray(u, dtype=np.float32)
    T, d1 = tab.shape
    e, p, ur = dyadic_index(T, u32.astype(np.float64))
    s = np.ldexp(ur, e + 1).astype(np.float32)  # exact
    c = tab[e]
    z = c[..., d1 - 1]
    for j in range(d1 - 2, -1, -1):
        z = fma_f32(z, s, c[..., j])
    if d1 == 1:
        z = fma_f32(np.float32(0.0), s, z)  # NaN input propagates
    z = np.where(p, z, -z).astype(np.float32)
    return z, e
