"""The benchmark's compact MLMC record (host logic only): per-level figures
for the configurations' estimators, surrogate fallbacks per level when any
step fell outside the trained range, zero fallback counts left out."""
import json
import math

from paper_2012_09715_amd import mlmc_driver as D


def _estimator(L, fallbacks):
    per_level = [{"level": l, "v_hat": 2.0 ** -(l + 3), "v2": 2.0 ** -(l + 3), "v4": 2.0 ** -(l + 20),
                  "c_hat_ns": 0.1 * 2 ** l, "c2_ns": 0.01 * 2 ** l, "c4_ns": 0.11 * 2 ** l,
                  "m_hat": 1000.5 / 2 ** l, "m_tilde": 900.2 / 2 ** l, "M_tilde": 3.1} for l in range(L + 1)]
    return {"eps": 1e-3, "levels": L, "formula_speedup": 22.41234, "measured_speedup": 0.98765,
            "theta_hat": 0.0388123, "se_hat": 7.1e-4, "theta_tilde": 0.039791, "se_tilde": 6.9e-4,
            "fallbacks": sum(fallbacks), "fallbacks_per_level": fallbacks, "per_level": per_level,
            "level_ms": {"exact": [1.0] * (L + 1)}}


def test_compact_record():
    full = {"cir": _estimator(2, [0, 5, 7]), "gbm_em": _estimator(2, [0, 0, 0]),
            "cir_poly1": _estimator(2, [0, 0, 0]), "fig4b_time_average": {"log2_ratio": {"em": [-1.0]}}}
    c = D.compact(full)
    assert "fig4b_time_average" not in c
    assert c["cir"]["per_level"]["fallbacks"] == [0, 5, 7] and c["cir"]["fallbacks"] == 12
    assert "fallbacks" not in c["gbm_em"] and "fallbacks" not in c["gbm_em"]["per_level"]
    assert "per_level" not in c["cir_poly1"] and "level_ms" not in c["cir_poly1"]
    pl = c["gbm_em"]["per_level"]
    assert pl["log2_v_hat"] == [-3.0, -4.0, -5.0] and pl["log2_v4"] == [-20.0, -21.0, -22.0]
    assert pl["m_hat"] == [math.ceil(1000.5), math.ceil(500.25), math.ceil(250.125)]
    assert c["cir"]["formula_speedup"] == 22.4 and c["cir"]["theta_hat"] == 0.03881
    json.dumps(c)  # plain JSON
