"""Coefficient tables of the two approximations, and their L2 errors (oracle).

Test infrastructure only.

Piecewise constant (Section 2.2, Theorem 2.3, Corollary 2.4): N = 2^q equal
intervals [k/N, (k+1)/N); the constant on interval k is one of
  E: the conditional mean E(Z | Phi(Z) in I_k)          (the paper's choice)
  C: Phi^-1 of the interval midpoint
  I: Phi^-1 of the endpoint nearer to 1/2 (the inner endpoint).
Because the integral of z phi(z) is -phi(z), the conditional mean is
N (phi(z_k) - phi(z_{k+1})) with z_k = Phi^-1(k/N) and phi(+-inf) = 0.

Dyadic piecewise polynomial (Section 2.3, Theorem 2.5 with r = 1/2; Section 3.3,
Table 1): a table of T entries serves u in (0, 1/2]:
  entry 0        u = 1/2 exactly, all coefficients zero (Section 3.3)
  entry e        the interval [2^-(e+1), 2^-e),  1 <= e <= T-2
  entry T-1      the singular interval (0, 2^-(T-1))
and u > 1/2 is served by antisymmetry.  On each interval the polynomial of
degree d is the L2 projection of Phi^-1 (the normal equations of the proof of
Theorem 2.5, generalised to degree d as the paper describes for piecewise
polynomials).  The polynomial is written in the local variable
s = u * 2^(e+1) (s in [1, 2), or (0, 2) on the singular interval); this only
changes the basis, not the approximant (see `to_u_monomials`).

Geometric intervals (Theorem 2.5 with a general decay rate r in (0, 1)): the
same layout with entry e on [B_e, B_(e-1)) and the singular (0, B_(T-2)), where
B_k is r^k / 2 computed by repeated FP64 multiplication and rounded to FP32
(the thresholds that decide the row, so that a FP32 input's row is fixed by
exact comparisons); the local variable is s = u / B_e.  r = 1/2 gives the
dyadic table (up to the rounding of the fit).
"""
import numpy as np
from scipy import integrate

from .normal import Phi, Phi_inv, phi

Z_FLOOR = -40.0  # Phi(-40) underflows to 0 in FP64


# --------------------------------------------------------------------------
# piecewise constant
# --------------------------------------------------------------------------
def const_table(n_intervals, construction="E"):
    """Constants Q_k on N equal intervals, k = 0..N-1 (Corollary 2.4)."""
    N = int(n_intervals)
    k = np.arange(N + 1, dtype=np.float64)
    edges = k / N
    if construction == "E":
        z = Phi_inv(edges)  # z_0 = -inf, z_N = +inf
        pz = phi(z)  # phi(+-inf) = 0
        return N * (pz[:-1] - pz[1:])
    if construction == "C":
        return Phi_inv((k[:-1] + 0.5) / N)
    if construction == "I":
        lo, hi = edges[:-1], edges[1:]
        inner = np.where(lo >= 0.5, lo, hi)
        return Phi_inv(inner)
    raise ValueError(construction)


def const_l2_error(Q):
    """RMSE ||Q - Phi^-1||_2 of a conditional-mean table by the projection
    identity ||Phi^-1 - Q||^2 = E(Z^2) - E(Q^2) = 1 - mean(Q_k^2), which holds
    because each Q_k is the L2 projection of Phi^-1 onto constants on I_k."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.sqrt(max(1.0 - np.mean(Q * Q), 0.0)))


def const_lp_error_quad(Q, p=2):
    """||Q - Phi^-1||_p by adaptive quadrature in z on every interval
    (Section 2.2, Theorem 2.3), u = Phi(z), du = phi(z) dz."""
    Q = np.asarray(Q, dtype=np.float64)
    N = len(Q)
    z = Phi_inv(np.arange(N + 1, dtype=np.float64) / N)
    z[0], z[-1] = Z_FLOOR, -Z_FLOOR
    total = 0.0
    for k in range(N):
        f = lambda t, c=Q[k]: abs(t - c) ** p * float(phi(t))
        val, _ = integrate.quad(f, z[k], z[k + 1], epsabs=0.0, epsrel=1e-12, limit=200)
        total += val
    return total ** (1.0 / p)


# --------------------------------------------------------------------------
# dyadic piecewise polynomial
# --------------------------------------------------------------------------
def dyadic_interval(e, n_entries):
    """(a, b, h): entry e covers u in [a, b) (or (0, b) for the singular
    entry), and s = u / h with h = 2^-(e+1) is the local variable."""
    T = int(n_entries)
    if not 1 <= e <= T - 1:
        raise ValueError("entry 0 is the u = 1/2 entry and has no interval")
    b = 2.0 ** (-e)
    a = 0.0 if e == T - 1 else 2.0 ** (-(e + 1))
    h = 2.0 ** (-(e + 1))
    return a, b, h


def _moment(j, a, b, h):
    """int_a^b s^j Phi^-1(u) du with s = u/h, by quadrature in z = Phi^-1(u):
    du = phi(z) dz, s = Phi(z)/h.  The integrand is smooth in z; the lower end
    z = -inf (a = 0) is truncated at -40 where phi underflows."""
    za = Z_FLOOR if a == 0.0 else float(Phi_inv(a))
    zb = float(Phi_inv(b))
    f = lambda z: (float(Phi(z)) / h) ** j * z * float(phi(z))
    # split the z-range so the quadrature sees the peak near zb
    pts = [zb - w for w in (8.0, 4.0, 2.0, 1.0, 0.5) if zb - w > za]
    edges = [za] + sorted(pts) + [zb]
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-13, limit=400)
        total += val
    return total


def dyadic_fit_entry(e, n_entries, degree):
    """Coefficients c_0..c_d (local variable s) of the L2-best polynomial of
    degree d on entry e: solve G c = m with G_ij = int s^(i+j) du and
    m_i = int s^i Phi^-1(u) du over the interval (the normal equations of
    Theorem 2.5's proof, in the basis 1, s, .., s^d)."""
    a, b, h = dyadic_interval(e, n_entries)
    d = int(degree)
    s0, s1 = a / h, b / h
    G = np.empty((d + 1, d + 1))
    for i in range(d + 1):
        for j in range(d + 1):
            p = i + j + 1
            G[i, j] = h * (s1 ** p - s0 ** p) / p  # int s^(i+j) du, du = h ds
    m = np.array([_moment(i, a, b, h) for i in range(d + 1)])
    return np.linalg.solve(G, m)


def dyadic_table(n_entries, degree):
    """T x (d+1) table in the local variable s; row 0 is all zeros
    (Section 3.3: u = 1/2 must map to Phi^-1(1/2) = 0)."""
    T, d = int(n_entries), int(degree)
    tab = np.zeros((T, d + 1))
    for e in range(1, T):
        tab[e] = dyadic_fit_entry(e, T, d)
    return tab


def to_u_monomials(coef_s, e):
    """Re-express a row c(s) = sum c_j s^j with s = u 2^(e+1) as sum a_j u^j,
    a_j = c_j 2^(j(e+1)): the basis Code 2 of the paper prints its
    coefficients in."""
    coef_s = np.asarray(coef_s, dtype=np.float64)
    return coef_s * 2.0 ** (np.arange(len(coef_s)) * (e + 1))


def singular_closed_form(b):
    """Intercept and gradient (in u) of the L2-best line on (0, b) in closed
    form (Section 2.3, proof of Theorem 2.5):
      alpha = 2 phi(z_b)/b - 3 Phi(sqrt2 z_b)/(b^2 sqrt(pi))
      beta  = 6/b^3 (Phi(sqrt2 z_b)/sqrt(pi) - b phi(z_b)),  z_b = Phi^-1(b)."""
    zb = float(Phi_inv(b))
    P2 = float(Phi(np.sqrt(2.0) * zb))
    pz = float(phi(zb))
    alpha = 2.0 * pz / b - 3.0 * P2 / (b * b * np.sqrt(np.pi))
    beta = 6.0 / b ** 3 * (P2 / np.sqrt(np.pi) - b * pz)
    return alpha, beta


def dyadic_l2_error(tab):
    """RMSE ||D - Phi^-1||_2 by the projection identity: on every interval D is
    the L2 projection of Phi^-1, so ||Phi^-1 - D||^2 = E(Z^2) - ||D||^2
    = 1 - 2 * sum_e int_{I_e} D^2 du (the factor 2 is the antisymmetric upper
    half).  int D^2 du is integrated exactly (polynomial in s)."""
    tab = np.asarray(tab, dtype=np.float64)
    T = tab.shape[0]
    tot = 0.0
    for e in range(1, T):
        a, b, h = dyadic_interval(e, T)
        sq = np.polynomial.polynomial.polymul(tab[e], tab[e])
        anti = np.polynomial.polynomial.polyint(sq)
        tot += h * (np.polynomial.polynomial.polyval(b / h, anti)
                    - np.polynomial.polynomial.polyval(a / h, anti))
    return float(np.sqrt(max(1.0 - 2.0 * tot, 0.0)))


def dyadic_l2_error_quad(tab):
    """Same RMSE by direct quadrature of (Phi^-1 - D)^2 over every interval in
    z (independent of the projection identity)."""
    tab = np.asarray(tab, dtype=np.float64)
    T = tab.shape[0]
    tot = 0.0
    for e in range(1, T):
        a, b, h = dyadic_interval(e, T)
        za = Z_FLOOR if a == 0.0 else float(Phi_inv(a))
        zb = float(Phi_inv(b))
        c = tab[e]
        f = lambda z: (z - np.polynomial.polynomial.polyval(float(Phi(z)) / h, c)) ** 2 * float(phi(z))
        pts = [zb - w for w in (8.0, 4.0, 2.0, 1.0, 0.5) if zb - w > za]
        edges = [za] + sorted(pts) + [zb]
        for lo, hi in zip(edges[:-1], edges[1:]):
            val, _ = integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-11, limit=400)
            tot += val
    return float(np.sqrt(2.0 * tot))


# --------------------------------------------------------------------------
# geometric intervals with a general decay rate r (Theorem 2.5)
# --------------------------------------------------------------------------
def geometric_thresholds(r, n_entries):
    """Interval bounds B_0..B_(T-1): b_0 = 1/2, b_k = b_(k-1) r by FP64
    multiplication, B_k = b_k rounded to FP32 (the thresholds that decide the
    row; exact powers of two when r = 1/2)."""
    T = int(n_entries)
    b = np.empty(T)
    b[0] = 0.5
    for k in range(1, T):
        b[k] = b[k - 1] * float(r)
    return b.astype(np.float32).astype(np.float64)


def geometric_interval(e, r, n_entries):
    """(a, b, h) of row e (1 <= e <= T-1): Theorem 2.5's I_e = [B_e, B_(e-1))
    for e < T-1 and the singular I_(T-1) = (0, B_(T-2)); s = t / h, h = B_e."""
    T = int(n_entries)
    if not 1 <= e <= T - 1:
        raise ValueError("row 0 is the u = 1/2 row and has no interval")
    B = geometric_thresholds(r, T)
    a = 0.0 if e == T - 1 else B[e]
    return a, B[e - 1], B[e]


def _legendre_moment(i, a, b):
    """int_a^b P_i(x) Phi^-1(u) du with x = (2u - a - b) / (b - a) mapping the
    interval onto [-1, 1], by quadrature in z = Phi^-1(u) as in `_moment`."""
    za = Z_FLOOR if a == 0.0 else float(Phi_inv(a))
    zb = float(Phi_inv(b))
    Pi = np.polynomial.legendre.Legendre.basis(i)
    f = lambda z: float(Pi((2.0 * float(Phi(z)) - a - b) / (b - a))) * z * float(phi(z))
    pts = [zb - w for w in (8.0, 4.0, 2.0, 1.0, 0.5) if zb - w > za]
    edges = [za] + sorted(pts) + [zb]
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        # for i >= 1 the moment is a small difference of large parts: an
        # absolute target keeps the coefficient error near 1e-15
        val, _ = integrate.quad(f, lo, hi, epsabs=1e-15 * (b - a), epsrel=1e-13, limit=400)
        total += val
    return total


def geometric_table(r, n_entries, degree):
    """T x (d+1) table of L2-best polynomials in s = t / B_e on the geometric
    intervals (row 0 all zeros, as for the dyadic tables, which it reproduces
    when r = 1/2).  The projection is taken in the Legendre basis of the
    interval, whose Gram matrix is diagonal (int_a^b P_i P_j du =
    (b - a) / (2i + 1) when i = j), and then written in powers of s: for r
    near 1 the normal equations in 1, s, .., s^d on the short range
    [1, 1/r) would be too ill-conditioned for FP64."""
    T, d = int(n_entries), int(degree)
    P = np.polynomial.polynomial
    tab = np.zeros((T, d + 1))
    for e in range(1, T):
        a, b, h = geometric_interval(e, r, T)
        leg = np.array([(2 * i + 1) / (b - a) * _legendre_moment(i, a, b) for i in range(d + 1)])
        px = np.polynomial.legendre.leg2poly(leg)           # powers of x
        x_of_s = np.array([-(a + b) / (b - a), 2.0 * h / (b - a)])  # x = (2 h s - a - b)/(b - a)
        cs = np.zeros(1)
        for k in range(len(px) - 1, -1, -1):                # Horner in the polynomial x(s)
            cs = P.polyadd(P.polymul(cs, x_of_s), [px[k]])
        tab[e, :len(cs)] = cs[: d + 1]
    return tab


def geometric_row(t, r, n_entries):
    """Row of the reflected t <= 1/2: 0 at t = 1/2, else the e with
    B_e <= t < B_(e-1) (e <= T-2) or the singular row T-1, decided by
    comparisons with the FP32 thresholds (no logarithm)."""
    t = np.asarray(t, float)
    B = geometric_thresholds(r, n_entries)
    T = int(n_entries)
    e = 1 + np.sum(t[..., None] < B[1:T - 1], axis=-1)
    return np.where(t >= 0.5, 0, e)


def geometric_transform(tab, r, u):
    """FP64 evaluation: reflect, row, s = t / B_e, Horner, sign."""
    u = np.asarray(u, float)
    T = tab.shape[0]
    B = geometric_thresholds(r, T)
    p = u < 0.5
    t = np.where(p, u, 1.0 - u)
    e = geometric_row(t, r, T)
    s = t / B[e]
    c = tab[e]
    z = np.zeros(u.shape)
    for j in range(c.shape[-1] - 1, -1, -1):
        z = z * s + c[..., j]
    return np.where(p, z, -z)


def geometric_l2_error(tab, r):
    """RMSE ||D - Phi^-1||_2 by the projection identity: on every interval the
    L2 fit D satisfies int D^2 = int D Phi^-1, so ||D - Phi^-1||^2 =
    1 - 2 sum_e int_(I_e) D^2 (both halves)."""
    T, d1 = tab.shape
    total = 0.0
    for e in range(1, T):
        a, b, h = geometric_interval(e, r, T)
        s0, s1 = a / h, b / h
        # int (sum c_j s^j)^2 du = h sum_ij c_i c_j (s1^(i+j+1) - s0^(i+j+1)) / (i+j+1)
        c = tab[e]
        for i in range(d1):
            for j in range(d1):
                p = i + j + 1
                total += c[i] * c[j] * h * (s1 ** p - s0 ** p) / p
    return float(np.sqrt(max(1.0 - 2.0 * total, 0.0)))
