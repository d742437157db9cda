"""Pins of oracle.prep (no GPU)."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.integrate import quad

from oracle import prep as P
from oracle.likelihood import trapezoid
from paper_2504_02034_amd import synth


def test_tangent_plane_is_gnomonic():
    rng = np.random.default_rng(3)
    ref = np.array([0.3, -0.5, 0.8]); ref /= np.linalg.norm(ref)
    th = np.arccos(ref[2]) + rng.normal(0, 0.05, 200)
    ph = math.atan2(ref[1], ref[0]) + rng.normal(0, 0.05, 200)
    x = P.tangent_plane(th, ph, ref)
    u = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    ang = np.arccos(np.clip(u @ ref, -1, 1))
    assert np.allclose(np.hypot(x[:, 0], x[:, 1]), np.tan(ang), rtol=1e-9, atol=1e-13)


def test_kde2d_is_scipy_scott():
    rng = np.random.default_rng(4)
    x = rng.multivariate_normal([0.01, -0.02], [[1e-3, 2e-4], [2e-4, 5e-4]], 3000)
    at = rng.normal(0, 0.03, (25, 2))
    ref = stats.gaussian_kde(x.T, bw_method="scott")(at.T)
    assert np.allclose(P.kde2d(x, at), ref, rtol=1e-12)


@pytest.mark.parametrize("mu,sig", [(0.5, 0.0011), (0.0015, 0.0011), (1.59, 0.002), (0.8, 0.09)])
def test_hat_integrals(mu, sig):
    grid = np.linspace(0.0, 1.6, 1000)
    j = P.hat_integrals(mu, sig, grid)
    dz = grid[1] - grid[0]
    # partition of unity of the hat basis on [z_lo, z_hi] (within the 8 sigma support)
    tot = (stats.norm.cdf(min(grid[-1], mu + 8 * sig), mu, sig)
           - stats.norm.cdf(max(grid[0], mu - 8 * sig), mu, sig))
    assert j.sum() == pytest.approx(tot, rel=1e-11)
    k0 = int(round((mu - grid[0]) / dz))
    for k in sorted({0, max(k0 - 1, 0), k0, min(k0 + 1, 999), 999}):
        a, b = grid[max(k - 1, 0)], grid[min(k + 1, 999)]
        hat = lambda z: max(0.0, 1.0 - abs(z - grid[k]) / dz)
        ref = quad(lambda z: hat(z) * stats.norm.pdf(z, mu, sig), a, b, points=[grid[k]],
                   epsabs=1e-15, epsrel=1e-12)[0]
        assert j[k] == pytest.approx(ref, rel=1e-8, abs=1e-13)


def test_hat_integrals_far_tail_mpmath():
    """Nodes 5-8 sigma from the mean: relative accuracy against 40-digit quadrature."""
    import mpmath
    mpmath.mp.dps = 40
    grid = np.linspace(0.0, 1.6, 1000)
    dz = grid[1] - grid[0]
    mu, sig = 0.70013, 0.0017
    j = P.hat_integrals(mu, sig, grid)
    for k in range(grid.size):
        u = abs(grid[k] - mu) / sig
        if not 5.0 <= u <= 7.0:
            continue
        f = lambda z: (max(0, 1 - abs(z - grid[k]) / dz)
                       * mpmath.exp(-(z - mu) ** 2 / (2 * sig ** 2)) / (sig * mpmath.sqrt(2 * mpmath.pi)))
        lo, hi = max(grid[k - 1], mu - 8 * sig), min(grid[k + 1], mu + 8 * sig)
        ref = mpmath.quad(f, [lo, grid[k], hi]) if lo < grid[k] < hi else mpmath.quad(f, [lo, hi])
        assert j[k] == pytest.approx(float(ref), rel=1e-11)


def test_catalog_normalisation_all_pixels():
    nside = 2
    rng = np.random.default_rng(5)
    n = 20000
    z = rng.uniform(0.0, 1.5, n)
    pix = rng.integers(0, synth.nside_npix(nside), n)
    grid = np.linspace(0.0, 1.6, 400)
    area = synth.pixel_area(nside)
    cat = P.catalog(z, pix, 0.001, grid, np.arange(synth.nside_npix(nside)), area)
    tau = trapezoid(grid)
    total = sum(area * np.sum(tau * r) for r in cat.rows.values())
    assert total == pytest.approx(1.0, rel=1e-12)
    assert np.allclose(area * sum(cat.rows.values()), cat.n_tot, rtol=1e-12, atol=0)
    assert np.sum(tau * cat.n_tot) == pytest.approx(1.0, rel=1e-12)


def test_region_covers_and_is_minimal():
    rng = np.random.default_rng(6)
    pix = rng.choice(np.arange(40), size=1000, p=np.arange(1, 41) / np.arange(1, 41).sum())
    reg = P.region(pix, 0.9)
    cov = np.isin(pix, reg).sum()
    assert cov >= 0.9 * pix.size
    counts = np.bincount(pix, minlength=40)
    # dropping the least-populated region pixel falls below 90%
    least = min(reg, key=lambda p: (counts[p], -p))
    assert cov - counts[least] < 0.9 * pix.size
