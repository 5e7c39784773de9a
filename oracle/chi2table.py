"""The paper's piecewise-polynomial approximation of the non-central
chi-squared inverse CDF (Section 5.1), in FP64 (oracle; test only).

Section 5.1 approximates the rescaled inverse
    P_nu(U; y) = (C_nu^-1(U; lambda) - lambda - nu) / (2 sqrt(lambda + nu)),
    y = nu / (lambda + nu) in (0, 1],
at a fixed nu by
  * two piecewise polynomials in U, one on (0, 1/2] and one on (1/2, 1) (the
    distribution is not antisymmetric), each on dyadic intervals of the
    distance t to the nearer end (t = U or t = 1 - U) as in Table 1:
    interval k = 1..K-1 is [2^-(k+1), 2^-k) and interval K the singular
    (0, 2^-K); the best L2 polynomial of degree d on each, in the local
    variable s = t 2^(k+1);
  * a set of such tables at knots equally spaced in sqrt(y), with
    y = 0 (the Gaussian limit P = Phi^-1(U)) and y = 1 (the central
    chi-squared, lambda = 0) as end knots, and linear interpolation in
    sqrt(y) between the two neighbouring knots.
The paper shows 8 intervals and 16 knots in its figure; its Table 6 errors
are reproduced with 15 intervals per half (the 16-row layout of the Gaussian
tables) and 16 knots, which is the reading used here (the tests pin it
against Table 6).  U = 1/2 belongs to the lower half's first interval.

The moments are integrated in t with Gauss-Legendre rules (t = b v^4 on the
singular interval), the exact P from scipy's non-central chi-squared
quantiles (ppf on the lower half, isf on the upper half).  Evaluation is in
FP64 and returns the formula value without clamping at 0.
"""
import numpy as np
from scipy import stats
from scipy.special import ndtri

N_KNOTS = 16
N_INTERVALS = 15


def _P_exact_t(t, upper, nu, lam):
    if lam == np.inf:
        z = ndtri(t)
        return -z if upper else z
    if lam > 0:
        x = stats.ncx2.isf(t, nu, lam) if upper else stats.ncx2.ppf(t, nu, lam)
    else:
        x = stats.chi2.isf(t, nu) if upper else stats.chi2.ppf(t, nu)
    s = lam + nu
    return (x - s) / (2.0 * np.sqrt(s))


def knot_lambda(nu, y):
    """lambda at a knot: y = nu / (lambda + nu); y = 0 is the Gaussian limit."""
    return np.inf if y == 0.0 else nu * (1.0 - y) / y


def fit_half(nu, lam, degree, upper, n_int=N_INTERVALS, n_gauss=80):
    """(n_int, d+1) coefficients in s = t 2^(k+1) for intervals k = 1..n_int."""
    gx, gw = np.polynomial.legendre.leggauss(n_gauss)
    d1 = degree + 1
    out = np.zeros((n_int, d1))
    for k in range(1, n_int + 1):
        b = 2.0 ** -k
        a = 0.0 if k == n_int else 2.0 ** -(k + 1)
        h = 2.0 ** -(k + 1)
        if a == 0.0:
            v = 0.5 * (gx + 1.0)
            t = b * v ** 4
            wt = 0.5 * gw * 4.0 * b * v ** 3
        else:
            t = a + (b - a) * 0.5 * (gx + 1.0)
            wt = 0.5 * gw * (b - a)
        P = _P_exact_t(t, upper, nu, lam)
        s = t / h
        G = np.array([[np.sum(wt * s ** (i + j)) for j in range(d1)] for i in range(d1)])
        m = np.array([np.sum(wt * s ** i * P) for i in range(d1)])
        out[k - 1] = np.linalg.solve(G, m)
    return out


def build(nu, degree, n_knots=N_KNOTS, n_int=N_INTERVALS):
    """Tables at the knots: array (n_knots, 2, n_int, d+1); [:, 0] lower half,
    [:, 1] upper half; knots sqrt(y_i) = i / (n_knots - 1)."""
    tab = np.zeros((n_knots, 2, n_int, degree + 1))
    for i in range(n_knots):
        y = (i / (n_knots - 1)) ** 2
        lam = knot_lambda(nu, y)
        tab[i, 0] = fit_half(nu, lam, degree, False, n_int)
        tab[i, 1] = fit_half(nu, lam, degree, True, n_int)
    return tab


def _eval_half(tab_half, t):
    """Polynomial of the dyadic interval of t (t in (0, 1/2])."""
    n_int = tab_half.shape[0]
    _, x = np.frexp(t)  # t = f 2^x, f in [1/2, 1) -> t in [2^(x-1), 2^x): interval k = -x
    k = np.clip(-x, 1, n_int)
    k = np.where(t == 0.0, n_int, k)
    s = np.ldexp(t, k + 1)
    c = tab_half[k - 1]
    z = np.zeros(t.shape)
    for j in range(c.shape[-1] - 1, -1, -1):
        z = z * s + c[..., j]
    return z


def _knot(nu, lam, n_knots):
    """Knot segment i and weight theta of sqrt(y) = sqrt(nu / (lambda + nu))."""
    q = np.sqrt(nu / (lam + nu))
    i = np.minimum(np.floor(q * (n_knots - 1)).astype(int), n_knots - 2)
    return i, q * (n_knots - 1) - i


def approx_P_half(tab, t, upper, lam, nu):
    """P~ on one half, given the tail distance t (U = t or U = 1 - t) and a
    scalar lambda."""
    i, th = _knot(nu, float(lam), tab.shape[0])
    side = 1 if upper else 0
    p0 = _eval_half(tab[i, side], t)
    p1 = _eval_half(tab[i + 1, side], t)
    return p0 + th * (p1 - p0)


def approx_P(tab, u, lam, nu):
    """P~(U; y(lambda)) by linear interpolation in sqrt(y) between the two
    neighbouring knots; U <= 1/2 uses the lower half (t = U), U > 1/2 the
    upper half (t = 1 - U)."""
    u = np.asarray(u, float)
    lam = np.broadcast_to(np.asarray(lam, float), u.shape)
    i, th = _knot(nu, lam, tab.shape[0])
    upper = u > 0.5
    t = np.where(upper, 1.0 - u, u)
    P = np.zeros(u.shape)
    for side in (0, 1):
        sel = upper if side else ~upper
        for kk in np.unique(i[sel]):
            s2 = sel & (i == kk)
            p0 = _eval_half(tab[kk, side], t[s2])
            p1 = _eval_half(tab[kk + 1, side], t[s2])
            P[s2] = p0 + th[s2] * (p1 - p0)
    return P


def approx_x(tab, u, lam, nu):
    """The approximate inverse lambda + nu + 2 sqrt(lambda + nu) P~ (no clamp)."""
    s = np.asarray(lam, float) + nu
    return s + 2.0 * np.sqrt(s) * approx_P(tab, u, lam, nu)


def l2_error(tab, nu, lam, n_panels=60, n_gauss=40):
    """||C~^-1(.; lambda) - C^-1(.; lambda)||_2 over U in (0, 1) (the RMSE of
    Table 6), by Gauss-Legendre quadrature on the dyadic panels
    [2^-(j+1), 2^-j] of t on each half (t > 2^-n_panels; the rest of the tail
    is below double precision)."""
    gx, gw = np.polynomial.legendre.leggauss(n_gauss)
    s = lam + nu
    total = 0.0
    for upper in (False, True):
        for j in range(1, n_panels):
            a, b = 2.0 ** -(j + 1), 2.0 ** -j
            t = a + (b - a) * 0.5 * (gx + 1.0)
            w = 0.5 * gw * (b - a)
            x = stats.ncx2.isf(t, nu, lam) if upper else stats.ncx2.ppf(t, nu, lam)
            xa = s + 2.0 * np.sqrt(s) * approx_P_half(tab, t, upper, lam, nu)
            total += np.sum(w * (xa - x) ** 2)
    return float(np.sqrt(total))
