"""Pins of the oracle's Phi^-1 (Section 2; Lemma 2.1 of Section 2.1)."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import ndtri

from oracle.normal import Phi, Phi_inv, phi


def test_against_mpmath_within_4_ulp():
    mp.mp.dps = 40
    rng = np.random.default_rng(11)
    u = np.concatenate([rng.random(200), 10.0 ** rng.uniform(-15, -1, 200),
                        0.5 - 2.0 ** -np.arange(2, 54), 0.5 + rng.uniform(-1e-9, 1e-9, 50)])
    z = Phi_inv(u)
    ref = np.array([float(mp.sqrt(2) * mp.erfinv(2 * mp.mpf(float(x)) - 1)) for x in u])
    ulps = np.abs(z - ref) / np.spacing(np.abs(ref))
    assert ulps.max() <= 4


def test_against_scipy_ndtri():
    # Cephes' ndtri (one of the library routines the paper names) is a
    # different method; both must agree to a few ulp.
    rng = np.random.default_rng(12)
    u = np.concatenate([rng.random(20000), 2.0 ** -rng.uniform(1, 1000, 2000)])
    z, r = Phi_inv(u), ndtri(u)
    assert np.all(np.abs(z - r) <= 8 * np.spacing(np.maximum(np.abs(r), 1e-300)) + 1e-300)


def test_antisymmetry_bitwise():
    rng = np.random.default_rng(13)
    u = rng.random(5000)
    v = 1.0 - u
    exact = (1.0 - v) == u  # 1-u exactly representable
    assert np.array_equal(Phi_inv(v)[exact], -Phi_inv(u)[exact])


def test_special_values():
    z = Phi_inv(np.array([0.5, 0.0, 1.0, np.nan, -0.1, 1.1]))
    assert z[0] == 0.0 and z[1] == -np.inf and z[2] == np.inf
    assert np.all(np.isnan(z[3:]))
    assert abs(Phi_inv(0.975) - 1.959963984540054) < 1e-15


def test_round_trip():
    # lower half only: Phi(z) near 1 is not resolved in FP64
    z = np.linspace(-37, 0, 1001)
    assert np.allclose(Phi_inv(Phi(z)), z, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("q", list(range(3, 54)))
def test_lemma_2_1_tail_bounds(q):
    # Lemma 2.1: z_q = Phi^-1(1 - 2^-q); 1 < 2^q phi(z_q)/z_q < (1 - z_q^-2)^-1,
    # and for q >= 10 the two square-root bounds.  The lemma says q >= 2, but
    # z_2 = 0.674 < 1 makes the upper bound negative; it holds from q = 3.
    zq = float(Phi_inv(1.0 - 2.0 ** -q))
    ratio = 2.0 ** q * float(phi(zq)) / zq
    assert 1.0 < ratio < 1.0 / (1.0 - zq ** -2)
    if q >= 10:
        lo = math.sqrt(q * math.log(4) - math.log(q * math.pi * (81 / 32) * math.log(4)))
        hi = math.sqrt(q * math.log(4))
        assert lo < zq < hi


def test_lemma_2_1_upper_bound_fails_at_q2():
    z2 = float(Phi_inv(1.0 - 2.0 ** -2))
    assert z2 < 1.0 and 1.0 / (1.0 - z2 ** -2) < 0.0
