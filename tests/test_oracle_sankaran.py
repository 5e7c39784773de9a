"""Pins of the oracle's Sankaran approximation (Section 5.1) against Table 6d
and against the reading of its Gaussian term."""
import numpy as np
import pytest
from scipy import stats

from oracle import normal, sankaran
from tests.conftest import read_golden

NUS = (1, 5, 10, 50, 100)


def _rows():
    return [(float(r[0]), r[1:]) for r in read_golden("table6d_sankaran_rmse.txt")]


@pytest.mark.slow
def test_table6d():
    # every printed entry, at nu = 5, 10, 50, 100 (nu = 1 below)
    for lam, row in _rows():
        for nu, want in zip(NUS[1:], row[1:]):
            got = sankaran.rmse_grid(nu, lam, lambda u: stats.ncx2.ppf(u, nu, lam), n_grid=50001)
            assert abs(got - float(want)) < 2.5e-3, (nu, lam, got, want)


def test_table6d_nu1_and_blanks():
    nu = 1
    ref = {lam: row[0] for lam, row in _rows()}
    for lam in (10.0, 50.0, 100.0, 200.0):
        got = sankaran.rmse_grid(nu, lam, lambda u: stats.ncx2.ppf(u, nu, lam), n_grid=50001)
        assert abs(got - float(ref[lam])) < 2.5e-3, (lam, got)
    # the blank entries: the clamp at 0 reaches into the body of the distribution
    for lam in (1.0, 5.0):
        assert ref[lam] == "-"
        u = np.linspace(1e-6, 1 - 1e-6, 20001)
        assert np.mean(sankaran.approx_x(u, nu, np.full(u.shape, lam)) == 0.0) > 1e-3


def test_printed_root_reading_is_rejected():
    # with the printed sqrt(2 c3) the error at nu = 50, lambda = 50 is ~1e1,
    # against 0.012 in Table 6d
    nu, lam = 50.0, 50.0
    c1, c2, c3 = sankaran.constants(nu, lam)
    u = np.linspace(1e-6, 1 - 1e-6, 20001)
    z = normal.Phi_inv(u)
    B = 1 + c1 * c2 * (c1 - 1 + 0.5 * (2 - c1) * c2 * c3) + c1 * np.sqrt(2 * c3) * (1 + 0.5 * c2 * c3) * z
    x_c3 = (nu + lam) * np.maximum(B, 0) ** (1 / c1)
    x = stats.ncx2.ppf(u, nu, lam)
    assert np.sqrt(np.mean((x_c3 - x) ** 2)) > 1.0
    assert np.sqrt(np.mean((sankaran.approx_x(u, nu, np.full(u.shape, lam)) - x) ** 2)) < 0.02


def test_limits():
    # lambda = 0: c1 = 1/3, c2 = 1/k, c3 = 0: the Wilson-Hilferty cube-root
    # normal approximation of the central chi-squared
    nu = 7.0
    c1, c2, c3 = sankaran.constants(nu, 0.0)
    assert np.isclose(c1, 1 / 3) and np.isclose(c2, 1 / nu) and c3 == 0.0
    u = np.array([0.1, 0.5, 0.9])
    z = normal.Phi_inv(u)
    wh = nu * (1 - 2 / (9 * nu) + z * np.sqrt(2 / (9 * nu))) ** 3
    assert np.allclose(sankaran.approx_x(u, nu, np.zeros(3)), wh, rtol=1e-14)
