"""Writes fig4b_derived.txt: the Figure 4b variance ratios
log2 Var(X_T - X~_T) / Var(X_T) of the CIR process (kappa = 1/2,
theta = xi = T = v0 = 1, nu = 2; Section 5.2) predicted from the chi-squared
tables' own errors (Section 5.1).  Calls only oracle/ (and scipy's
non-central chi-squared quantiles through oracle/chi2table.py).

Level 0 (one transition of the whole horizon): X_T = c x(U), X~_T = c x~(U),
so the ratio is exactly Var_U(x - x~) / (2 (nu + 2 lambda_0)), the variance
of chi^2_nu(lambda_0) being 2 (nu + 2 lambda_0); the U-integral runs over
t = min(U, 1-U) in [2^-24, 1/2] (the u24 grid's range) by Gauss-Legendre
panels on the dyadic intervals.
Many levels (lambda_n -> infinity): the table tends to its y = 0 knot, the
16-row normal table, with x - x~ = 2 sqrt(lambda + nu) (P - P~); a
perturbation of step n reaches X_T damped by e^(-kappa (T - t_n)), and
4 c (lambda_n + nu) -> xi^2 delta v_n, so
Var(X_T - X~_T) -> xi^2 E(P - P~)^2 int_0^T E(v_t) e^(-2 kappa (T - t)) dt,
which for v0 = theta equals E(P - P~)^2 Var(v_T): the ratio tends to the
normal table's mean-square error (on the u24 grid, as in table3_derived.txt).

    python tests/golden/make_fig4b_derived.py
"""
import os
import sys

import numpy as np
from scipy import stats

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import chi2table as ct  # noqa: E402
from oracle import tables  # noqa: E402
from oracle.dtypes import round_f32  # noqa: E402
from oracle.normal import Phi_inv  # noqa: E402
from oracle.transform import dyadic_transform_f32  # noqa: E402

NU = 2.0
KAPPA, THETA, XI, T, V0 = 0.5, 1.0, 1.0, 1.0, 1.0


def level0_ratio(tab):
    c = XI ** 2 * (1.0 - np.exp(-KAPPA * T)) / (4.0 * KAPPA)
    lam = V0 * np.exp(-KAPPA * T) / c
    s = lam + NU
    gx, gw = np.polynomial.legendre.leggauss(40)
    m1 = m2 = 0.0
    for upper in (False, True):
        for j in range(1, 24):
            a, b = 2.0 ** -(j + 1), 2.0 ** -j
            t = a + (b - a) * 0.5 * (gx + 1.0)
            w = 0.5 * gw * (b - a)
            x = stats.ncx2.isf(t, NU, lam) if upper else stats.ncx2.ppf(t, NU, lam)
            xa = np.maximum(s + 2.0 * np.sqrt(s) * ct.approx_P_half(tab, t, upper, lam, NU), 0.0)
            d = x - xa
            m1 += np.sum(w * d)
            m2 += np.sum(w * d * d)
    return np.log2((m2 - m1 * m1) / (2.0 * (NU + 2.0 * lam))), lam


def main():
    u = (np.arange(1 << 23, dtype=np.float64) + 0.5) * 2.0 ** -23
    z = Phi_inv(u)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fig4b_derived.txt")
    lines = []
    for deg, name in ((1, "linear"), (3, "cubic")):
        r0, lam0 = level0_ratio(ct.build(NU, deg))
        za = dyadic_transform_f32(round_f32(tables.dyadic_table(16, deg)), u.astype(np.float32))[0]
        rinf = np.log2(np.mean((za.astype(np.float64) - z) ** 2))
        lines.append(f"{name} {r0:.3f} {rinf:.3f}")
    with open(out, "w") as f:
        f.write("# Figure 4b (nu = 2): log2 Var(X - X~)/Var(X) predicted from the tables' errors\n")
        f.write(f"# (written by make_fig4b_derived.py; lambda_0 = {lam0:.6f})\n")
        f.write("# table level0 large_level_limit\n")
        f.write("\n".join(lines) + "\n")
    print(open(out).read())


if __name__ == "__main__":
    main()
