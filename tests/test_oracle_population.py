"""Pins of oracle.population (no GPU)."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.integrate import quad

from oracle.population import mass_weight, p_m1, p_m2_given_m1, psi

SETS = [(3.4, 5.0, 87.0, 34.0, 3.6, 0.04), (1.0, 5.0, 87.0, 34.0, 3.6, 0.5),
        (12.0, 3.0, 150.0, 60.0, 9.0, 0.99), (1.5, 7.0, 50.0, 2.0, 0.4, 0.2)]


@pytest.mark.parametrize("p", SETS)
def test_m1_normalised(p):
    alpha, mmin, mmax, mu, sg, lg = p
    f = lambda m: float(p_m1(m, alpha, mmin, mmax, mu, sg, lg))
    pts = [x for x in (mu - 3 * sg, mu, mu + 3 * sg) if mmin < x < mmax]
    val = quad(f, mmin, mmax, points=pts, limit=400, epsabs=0, epsrel=1e-12)[0]
    assert val == pytest.approx(1.0, rel=1e-10)


@pytest.mark.parametrize("beta", [1.1, -1.0, -4.0, 12.0, 0.0])
@pytest.mark.parametrize("m1", [6.0, 34.0, 87.0])
def test_m2_normalised(beta, m1):
    val = quad(lambda m: float(p_m2_given_m1(m, m1, beta, 5.0)), 5.0, m1, epsrel=1e-12)[0]
    assert val == pytest.approx(1.0, rel=1e-10)


def test_limits_continuous():
    m = np.array([5.5, 20.0, 80.0])
    a1 = p_m1(m, 1.0, 5, 87, 34, 3.6, 0.0)
    assert np.allclose(p_m1(m, 1.0 + 1e-7, 5, 87, 34, 3.6, 0.0), a1, rtol=1e-6)
    b1 = p_m2_given_m1(m, 85.0, -1.0, 5.0)
    assert np.allclose(p_m2_given_m1(m, 85.0, -1.0 + 1e-7, 5.0), b1, rtol=1e-6)


def test_peak_is_truncnorm():
    m = np.linspace(5, 87, 41)
    ref = stats.truncnorm.pdf(m, (5 - 34) / 3.6, (87 - 34) / 3.6, loc=34, scale=3.6)
    assert np.allclose(p_m1(m, 3.4, 5, 87, 34, 3.6, 1.0), ref, rtol=1e-12)


def test_power_law_is_truncpareto():
    m = np.linspace(5, 87, 41)
    ref = stats.truncpareto.pdf(m, 3.4 - 1.0, 87 / 5, scale=5.0)
    assert np.allclose(p_m1(m, 3.4, 5, 87, 34, 3.6, 0.0), ref, rtol=1e-12)


def test_support_is_hard():
    lam = np.array([70, .3, 1, 1.91, 3.4, 1.1, 5, 87, 34, 3.6, .04, 2.7, 3, 2])
    m1 = np.array([4.999, 5.0, 30.0, 87.0, 87.001, 30.0])
    m2 = np.array([4.0, 5.0, 30.0, 5.0, 6.0, 30.0001])
    w = mass_weight(m1, m2, lam)
    assert w[0] == 0 and w[4] == 0 and w[5] == 0
    assert w[2] > 0 and w[3] > 0
    assert w[1] == 0       # m1 = mmin: the secondary's support is empty


def test_rate_shape_values():
    g, k, zp = 2.7, 3.0, 2.0
    assert psi(0.0, g, k, zp) == pytest.approx(1.0 / (1.0 + 3.0 ** (-(g + k))), rel=1e-15)
    assert psi(zp, g, k, zp) == pytest.approx(3.0 ** g / 2.0, rel=1e-15)
    z = 1e4
    assert psi(z, g, k, zp) == pytest.approx((1 + z) ** (-k) * 3.0 ** (g + k), rel=1e-6)
