"""Pins of the oracle's 3D kernel (Sect. 2.2: one Gaussian KDE of the samples
in redshift and sky, evaluated at the pixel centres), no GPU: the bandwidth
matrix and kernel values against scipy.stats.gaussian_kde in 3-D, the
truncated sums against the dense ones on correlated data (the conditional
shift and width that place the windows), and the sky marginal on a flat
catalogue row; through ln L on the 10-event data."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import likelihood as L
from paper_2504_02034_amd import synth

LAM = synth.LAMBDA_TRUTH.copy()


def correlated_samples(n=300, seed=4):
    """z correlated with the sky offset u, so that B != 0."""
    rng = np.random.default_rng(seed)
    u = rng.normal(0.0, 0.01, n)
    v = rng.normal(0.0, 0.012, n) + 0.4 * u
    z = 0.7 + 3.0 * u + rng.normal(0.0, 0.02, n)
    w = rng.gamma(3.0, 1.0, n)
    return z, u, v, w


def test_bandwidth_and_values_are_scipys():
    z, u, v, w = correlated_samples()
    H = L.kde3d_bandwidth(z, u, v, w)
    kde = stats.gaussian_kde(np.stack([z, u, v]), weights=w)
    assert np.allclose(H, kde.covariance, rtol=1e-12, atol=0)
    grid = np.linspace(0.4, 1.0, 601)
    tau = L.trapezoid(grid)
    row = 1.0 + 0.5 * np.sin(7.0 * grid)
    gz = np.exp(-grid)
    for uk, vk in ((0.0, 0.0), (0.006, -0.004), (-0.01, 0.015)):
        I, s = L.event_integral_3d(z, w, u, v, [(uk, vk)], [2.5e-4], [row], grid, tau, gz, None)
        pts = np.stack([grid, np.full(grid.size, uk), np.full(grid.size, vk)])
        ref = 2.5e-4 * np.sum(tau * row * gz * kde(pts) * w.sum() / z.size)
        assert I == pytest.approx(ref, rel=1e-12)


def test_truncated_sums_equal_the_dense_ones():
    """With T = 8.6 every dropped term is below e^-37 of its peak: on data
    whose redshift follows the sky offset the windows sit at the conditional
    mean, so truncated and dense agree to rounding."""
    z, u, v, w = correlated_samples(500, 5)
    grid = np.linspace(0.0, 1.6, 2001)
    tau = L.trapezoid(grid)
    rows = [np.exp(-0.5 * ((grid - c) / 0.05) ** 2) + 0.01 for c in (0.65, 0.72)]
    uv = [(0.004, 0.002), (-0.012, -0.006)]
    gz = 1.0 / (1.0 + grid) ** 3
    dense, s0 = L.event_integral_3d(z, w, u, v, uv, [1e-4, 1e-4], rows, grid, tau, gz, None)
    trunc, s1 = L.event_integral_3d(z, w, u, v, uv, [1e-4, 1e-4], rows, grid, tau, gz, 8.6)
    assert s0 == s1
    assert trunc == pytest.approx(dense, rel=1e-12)
    # a window placed without the shift B dO would cut the kernel: check that
    # the shift is material here (several conditional widths across the pixels)
    H = L.kde3d_bandwidth(z, u, v, w)
    B = H[0, 1:] @ np.linalg.inv(H[1:, 1:])
    assert abs(B @ np.array(uv[0]) - B @ np.array(uv[1])) > 3 * s0


def test_sky_marginal_on_a_flat_row():
    """n = 1 and g = 1 on a grid wide and fine enough for the redshift part to
    integrate to 1: I = area (1/N) sum_j w_j N2(centre - (u_j, v_j); H_OO)."""
    z, u, v, w = correlated_samples(200, 6)
    grid = np.linspace(-0.5, 2.0, 25001)
    tau = L.trapezoid(grid)
    H = L.kde3d_bandwidth(z, u, v, w)
    for uk, vk in ((0.0, 0.0), (0.01, 0.01)):
        I, _ = L.event_integral_3d(z, w, u, v, [(uk, vk)], [1.0], [np.ones(grid.size)], grid, tau,
                                   np.ones(grid.size), None)
        n2 = stats.multivariate_normal(mean=[0.0, 0.0], cov=H[1:, 1:])
        ref = np.sum(w * n2.pdf(np.stack([uk - u, vk - v], axis=1))) / z.size
        assert I == pytest.approx(ref, rel=1e-9)


def test_degenerate_weights_give_zero():
    z, u, v, w = correlated_samples(50, 7)
    w0 = np.zeros_like(w)
    w0[3] = 1.0
    grid = np.linspace(0.0, 1.6, 101)
    I, s = L.event_integral_3d(z, w0, u, v, [(0.0, 0.0)], [1.0], [np.ones(101)], grid,
                               L.trapezoid(grid), np.ones(101), 8.6)
    assert I == 0.0 and math.isnan(s)


@pytest.fixture(scope="module")
def small_data():
    from tests.datasets import small
    return small()


def test_through_ln_l(small_data):
    d = small_data
    ev = d.o_events[:3]
    a = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=8.6, kernel="3d")
    b = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=8.6, kernel="many1d")
    print("3d", a["lnI"], "many1d", b["lnI"])
    assert np.all(np.isfinite(a["lnI"]))
    assert np.all(np.abs(a["lnI"] - b["lnI"]) < 1.0)
    with pytest.raises(ValueError):
        L.lnl(ev, d.o_cat, d.o_inj, LAM, kernel="3d", shape="epanechnikov")
