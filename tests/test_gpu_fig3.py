"""Figure 3 and Table 3 of Section 4.1 on the device: GBM with P = X_T, the
two-way variance v^_l of the exact levels and the four-way variance V~_l of
the correction levels for Rademacher, constant-1024, linear-16 and cubic-16
approximations, Euler-Maruyama and Milstein, levels 0..10, 2^20 paths per
level and kind.

Pins: v^_l falls as 2^-l (Euler-Maruyama, strong order 1/2) and 2^-2l
(Milstein, strong order 1); Table 3's drops log2(V~/v^) (Euler-Maruyama)
within 1.5 of the printed -1 / -13 / -14 and of the prediction from each
table's own mean-square error (tests/golden/table3_derived.txt; for the cubic
table the prediction, -21.9, not the printed -25, which leaves out the
singular intervals); with Milstein the four-way variances of the constant,
linear and cubic tables fall as 2^-2l too (Figure 3b: the lines run parallel).
"""
import numpy as np
import pytest

from paper_2012_09715_amd import mlmc_driver as D
from tests.conftest import read_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def study():
    return D.fig3_study()


def slope(levels, y):
    return np.polyfit(levels, y, 1)[0]


def test_two_way_variance_slopes(study):
    lv = np.array(study["levels"])
    sel = lv >= 3
    em = np.array(study["em"]["log2_v_hat"])
    mil = np.array(study["milstein"]["log2_v_hat"])
    assert -1.2 < slope(lv[sel], em[sel]) < -0.8, em
    assert -2.2 < slope(lv[sel], mil[sel]) < -1.8, mil


def test_table3_drops(study):
    pred = {r[0]: float(r[2]) for r in read_golden("table3_derived.txt")}
    printed = {"rademacher": -1.0, "const1024": -13.0, "linear16": -14.0}
    drops = study["em"]["drop"]
    for name, d in drops.items():
        assert abs(d - pred[name]) <= 1.5, (name, d, pred[name])
        if name in printed:
            assert abs(d - printed[name]) <= 1.5, (name, d, printed[name])
    # level by level the drop stays put (Figure 3a: parallel lines)
    lv = np.array(study["levels"])
    vh = np.array(study["em"]["log2_v_hat"])
    for name in ("const1024", "linear16", "cubic16"):
        r = np.array(study["em"]["log2_V4"][name])[lv >= 1] - vh[lv >= 1]
        assert r.max() - r.min() < 3.0, (name, r)


def test_milstein_four_way_slopes(study):
    lv = np.array(study["levels"])
    sel = lv >= 2
    for name in ("const1024", "linear16", "cubic16"):
        v4 = np.array(study["milstein"]["log2_V4"][name])
        assert -2.5 < slope(lv[sel], v4[sel]) < -1.5, (name, v4)
