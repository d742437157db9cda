"""Pins of oracle.cosmology against closed forms, high-precision quadrature
and a number printed in the paper (no GPU)."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import cosmology as C
from oracle.population import psi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("z", [0.01, 0.3, 1.0, 1.3, 4.0, 24.9])
def test_einstein_de_sitter_closed_form(z):
    # Om = 1: chi = 2 (1 - 1/sqrt(1+z))
    h0 = 70.0
    s = math.sqrt(1 + z)
    exact = 2.0 * C.C_KM_S / h0 * (1 + z) * z / (s * (s + 1))     # 1 - 1/s without cancellation
    assert C.dl_em(z, h0, 1.0) == pytest.approx(exact, rel=1e-14)


def test_empty_universe_limit():
    z = np.linspace(0, 25, 101)
    assert np.allclose(C.chi(z, 0.0), z, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("om", [0.1, 0.3, 0.5])
@pytest.mark.parametrize("z", [0.1, 0.5, 1.0, 1.5, 10.0, 25.0])
def test_chi_vs_mpmath(om, z):
    mpmath.mp.dps = 30
    ref = mpmath.quad(lambda t: 1 / mpmath.sqrt(om * (1 + t) ** 3 + 1 - om), [0, z])
    assert float(C.chi(z, om)) == pytest.approx(float(ref), rel=2e-15)


@pytest.mark.parametrize("lam", [(70, 0.3, 1.0, 1.91), (40, 0.1, 0.3, 10.0),
                                 (140, 0.5, 3.0, 0.5), (67, 0.3, 1.8, 2.7)])
def test_derivative_vs_richardson(lam):
    z = np.array([0.05, 0.4, 1.2, 3.0, 12.0])
    f = lambda zz: C.dl_gw(zz, *lam)
    def cd(h):
        return (f(z + h) - f(z - h)) / (2 * h)
    h = 1e-3
    rich = (4 * cd(h / 2) - cd(h)) / 3
    assert np.allclose(C.ddl_gw_dz(z, *lam), rich, rtol=1e-10)


def test_gr_limit_is_bitwise():
    z = np.linspace(0.0, 3.0, 301)
    assert np.array_equal(C.dl_gw(z, 70, 0.3, 1.0, 7.3), C.dl_em(z, 70, 0.3))
    assert np.array_equal(C.ddl_gw_dz(z, 70, 0.3, 1.0, 7.3), C.ddl_gw_dz(z, 70, 0.3, 1.0, 0.2))
    d = np.array([10.0, 800.0, 5000.0, 20000.0])
    assert np.array_equal(C.invert_dl(d, 70, 0.3, 1.0, 7.3), C.invert_dl(d, 70, 0.3, 1.0, 0.0))


def test_xi_limits():
    z = np.array([0.0, 1.0, 1e6])
    x = C.xi(z, 1.8, 2.0)
    assert x[0] == 1.0 and x[2] == pytest.approx(1.8, rel=1e-11)
    assert np.allclose(C.xi(z, 1.8, 0.0), 1.0, rtol=0, atol=2.3e-16)


def test_inversion_eds_closed_form():
    # Om = 1: d = (2c/H0)(s^2 - s), s = sqrt(1+z)  =>  s = (1 + sqrt(1 + 2 d H0/c)) / 2
    h0 = 70.0
    d = np.array([1.0, 50.0, 700.0, 6710.42513668539, 25000.0])
    x = 2 * d * h0 / C.C_KM_S
    sm1 = x / (2 * (np.sqrt(1 + x) + 1))           # s - 1 without cancellation
    assert np.allclose(C.invert_dl(d, h0, 1.0, 1.0, 0.0), sm1 * (sm1 + 2), rtol=1e-14, atol=0)


@pytest.mark.parametrize("lam", [(70, 0.3, 1.0, 1.91), (20, 0.45, 0.3, 10.0), (140, 0.1, 3.0, 0.0)])
def test_inversion_roundtrip(lam):
    rng = np.random.default_rng(1)
    d = np.exp(rng.uniform(0, math.log(3e4), 2000))
    z = C.invert_dl(d, *lam)
    ok = np.isfinite(z)
    assert np.all(ok | (d > C.dl_gw(C.Z_MAX, *lam)))
    assert np.allclose(C.dl_gw(z[ok], *lam), d[ok], rtol=2e-15)


def test_nonmonotone_detected():
    with pytest.raises(C.NonMonotone):
        C.invert_dl(np.array([100.0]), 70, 0.3, 0.02, 20.0)


def test_paper_merger_count():
    """Sect. 3.3: ~1.4e4 events/yr to z=1.3 (printed to two digits)."""
    g = json.load(open(os.path.join(GOLDEN, "merger_count.json")))
    p = g["params"]
    from scipy.integrate import quad
    f = lambda z: (psi(z, p["gamma"], p["kappa"], p["z_p"]) / (1 + z)
                   * C.comoving_volume_element(z, p["H0"], p["Om"]) / 1e9)
    val = p["R0_per_Gpc3_yr"] * quad(f, 0, p["z_max"], epsrel=1e-12)[0]
    lo = g["printed_value"] - 0.05e4
    hi = g["printed_value"] + 0.05e4
    assert lo <= val <= hi, val
    # and with the rate normalised to psi(0) = 1
    val0 = val / float(psi(0.0, p["gamma"], p["kappa"], p["z_p"]))
    assert lo <= val0 <= hi, val0
