"""Nested MLMC cost, optimal allocation and savings (oracle; test only).

Section 4.1.  For the regular estimator with per-level variances v^_l and
costs c^_l, and the nested estimator with two-way (v~_l, c~_l) and four-way
(V~_l, C~_l) terms, at target MSE eps^2 with variance eps^2 / 2:
  T^ = 2 eps^-2 (sum_l sqrt(v^_l c^_l))^2
  T~ = 2 eps^-2 (sum_l sqrt(v~_l c~_l) + sqrt(V~_l C~_l))^2
  m^_l = eps^-1 sqrt(2 T^ v^_l / c^_l),  m~_l = eps^-1 sqrt(2 T~ v~_l / c~_l),
  M~_l = eps^-1 sqrt(2 T~ V~_l / C~_l)
and the savings bound T~ <= T^ max_l (v~ c~ / v^ c^)(1 + sqrt(V~ C~ / v~ c~))^2.
"""
import numpy as np


def total_cost(eps, v, c):
    v, c = np.asarray(v, float), np.asarray(c, float)
    return 2.0 * eps ** -2 * np.sum(np.sqrt(v * c)) ** 2


def nested_total_cost(eps, v2, c2, v4, c4):
    v2, c2, v4, c4 = (np.asarray(a, float) for a in (v2, c2, v4, c4))
    return 2.0 * eps ** -2 * np.sum(np.sqrt(v2 * c2) + np.sqrt(v4 * c4)) ** 2


def paths(eps, T, v, c):
    return eps ** -1 * np.sqrt(2.0 * T * np.asarray(v, float) / np.asarray(c, float))


def allocation(eps, vh, ch, v2, c2, v4, c4):
    """Returns dict with T_hat, T_tilde, m_hat, m_tilde, M_tilde, speedup."""
    Th = total_cost(eps, vh, ch)
    Tt = nested_total_cost(eps, v2, c2, v4, c4)
    return {"T_hat": Th, "T_tilde": Tt,
            "m_hat": paths(eps, Th, vh, ch),
            "m_tilde": paths(eps, Tt, v2, c2),
            "M_tilde": paths(eps, Tt, v4, c4),
            "speedup": Th / Tt}


def savings_bound(vh, ch, v2, c2, v4, c4):
    vh, ch, v2, c2, v4, c4 = (np.asarray(a, float) for a in (vh, ch, v2, c2, v4, c4))
    r = (v2 * c2) / (vh * ch) * (1.0 + np.sqrt((v4 * c4) / (v2 * c2))) ** 2
    return float(np.max(r))


def table3_row(log2_var_ratio, cost_ratio):
    """Savings under the paper's simplifications for its Tables 3 and 7:
    v~ = v^, C~ = c^ + c~, the same ratios on every level.  Returns
    (speedup, efficiency, m~/m^, m~/M~)."""
    ch, ct = float(cost_ratio), 1.0
    vh = 1.0
    V = 2.0 ** log2_var_ratio
    Ct = ch + ct
    r = allocation(1.0, [vh], [ch], [vh], [ct], [V], [Ct])
    sp = r["speedup"]
    return sp, sp / cost_ratio, float(r["m_tilde"][0] / r["m_hat"][0]), float(r["m_tilde"][0] / r["M_tilde"][0])
