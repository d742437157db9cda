"""Pins of the oracle's kernel options (Sect. 2.3: Gaussian or Epanechnikov
1-D kernels, binned data sets), no GPU: the Epanechnikov kernel against
scikit-learn's and its normalisation and variance on a fine grid; the binned
data set against the unbinned one when every weighted sample sits at a bin
centre, its weight total, its error within the half-bin shift bound and the
degenerate
one-redshift case; the kernel options through ln L (the reduction of
single-1D to many-1D with identical pixels holds for every option)."""
import copy
import math

import numpy as np
import pytest

from oracle import likelihood as L
from paper_2504_02034_amd import synth

LAM = synth.LAMBDA_TRUTH.copy()


def test_epanechnikov_is_scikit_learns():
    from sklearn.neighbors import KernelDensity
    rng = np.random.default_rng(3)
    z = rng.normal(0.9, 0.05, 400)
    w = rng.gamma(2.0, 1.0, 400)
    h = 0.013
    grid = np.linspace(0.6, 1.2, 777)
    ours = (w @ L.kernel_values(grid, z, h, "epanechnikov")) / w.sum()
    kd = KernelDensity(kernel="epanechnikov", bandwidth=math.sqrt(5.0) * h)
    kd.fit(z[:, None], sample_weight=w)
    ref = np.exp(kd.score_samples(grid[:, None]))
    pos = ref > 1e-12
    assert np.allclose(ours[pos], ref[pos], rtol=1e-10, atol=0)
    assert np.all(ours[~pos] < 1e-10)


@pytest.mark.parametrize("zj,h", [(0.7345, 0.02), (1.1, 0.0071)])
def test_epanechnikov_mass_and_variance(zj, h):
    """Trapezoid on a fine grid: mass 1, mean z_j, variance h^2 (the scale
    a = sqrt(5) is what makes the variance h^2)."""
    grid = np.linspace(0.0, 2.0, 200_001)
    tau = L.trapezoid(grid)
    k = L.kernel_values(grid, [zj], h, "epanechnikov")[0]
    assert np.sum(tau * k) == pytest.approx(1.0, abs=1e-7)
    assert np.sum(tau * k * grid) == pytest.approx(zj, abs=2e-5 * h)
    assert np.sum(tau * k * (grid - zj) ** 2) == pytest.approx(h * h, rel=1e-6)
    assert np.all(k[np.abs(grid - zj) >= math.sqrt(5.0) * h] == 0.0)
    assert k.max() == pytest.approx(0.75 / (math.sqrt(5.0) * h), rel=1e-6)


def _kde(grid, z, w, h, shape):
    return w @ L.kernel_values(grid, z, h, shape)


@pytest.mark.parametrize("shape", ["gaussian", "epanechnikov"])
def test_binned_equals_unbinned_at_bin_centres(shape):
    """Zero-weight samples at both ends fix the bin range; every weighted
    sample at a bin centre: the binned data set is the samples themselves."""
    rng = np.random.default_rng(5)
    nb, lo, hi = 12, 0.41, 0.77
    k = rng.integers(0, nb, 40)
    zc = lo + (k + 0.5) * ((hi - lo) / nb)
    z = np.concatenate([[hi, lo], zc])
    w = np.concatenate([[0.0, 0.0], rng.uniform(0.1, 2.0, 40)])
    grid = np.linspace(0.2, 1.0, 801)
    bz, bw = L.bin_samples(z, w, nb)
    assert bz.size == nb and bw.sum() == pytest.approx(w.sum(), rel=1e-15)
    a = _kde(grid, bz, bw, 0.03, shape)
    b = _kde(grid, z, w, 0.03, shape)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * b.max())


def test_binning_error_within_the_shift_bound():
    """Gaussian KDE of 2000 samples: binning moves each sample by at most half
    a bin width, so the KDE moves by at most sum w max|K'| width / 2, with
    max|K'| = 1 / (h^2 sqrt(2 pi e)); the error falls as the bins narrow."""
    rng = np.random.default_rng(6)
    z = rng.normal(0.8, 0.06, 2000)
    w = rng.uniform(0.5, 1.5, 2000)
    grid = np.linspace(0.5, 1.1, 601)
    h = 0.02
    exact = _kde(grid, z, w, h, "gaussian")
    slope = 1.0 / (h * h * math.sqrt(2.0 * math.pi * math.e))
    errs = []
    for nb in (16, 32, 64, 128):
        bz, bw = L.bin_samples(z, w, nb)
        width = (z.max() - z.min()) / nb
        err = np.max(np.abs(_kde(grid, bz, bw, h, "gaussian") - exact))
        assert err <= w.sum() * slope * width / 2
        assert np.all(np.abs(bz - np.round((bz - z.min()) / width - 0.5) * width - z.min()
                             - width / 2) < 1e-12)
        errs.append(err)
    print("errors", errs)
    assert np.all(np.diff(errs) < 0)
    assert errs[-1] < 4e-3 * exact.max()


def test_binning_degenerate_cases():
    bz, bw = L.bin_samples(np.full(5, 0.3), np.arange(1.0, 6.0), 8)
    assert bw[0] == 15.0 and np.all(bw[1:] == 0.0) and np.all(bz == 0.3)
    bz, bw = L.bin_samples(np.array([0.2, 0.6]), np.array([1.0, 3.0]), 4)
    assert np.array_equal(bw, [1.0, 0.0, 0.0, 3.0])
    assert np.allclose(bz, [0.25, 0.35, 0.45, 0.55], rtol=1e-15)


@pytest.fixture(scope="module")
def small_data():
    from tests.datasets import small
    return small()


@pytest.mark.parametrize("shape,n_bins", [("epanechnikov", 0), ("gaussian", 16),
                                          ("epanechnikov", 16)])
def test_options_reduce_single1d_to_many1d(small_data, shape, n_bins):
    d = small_data
    ev = copy.deepcopy(d.o_events[:4])
    for e in ev:
        p0 = e.pixels[0]
        for px in e.pixels[1:]:
            px.dl, px.m1d, px.m2d = p0.dl.copy(), p0.m1d.copy(), p0.m2d.copy()
        for px in e.pixels:
            px.s = None
        e.samples = None
    a = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=8.6, kernel="single1d", shape=shape, n_bins=n_bins)
    b = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=8.6, kernel="many1d", shape=shape, n_bins=n_bins)
    assert np.all(np.isfinite(a["lnI"]))
    assert np.allclose(a["lnI"], b["lnI"], rtol=1e-12, atol=0)
    plain = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=8.6, kernel="single1d")
    assert np.max(np.abs(a["lnI"] - plain["lnI"])) > 1e-8


def test_options_change_ln_i_a_little(small_data):
    """The options are different estimators of the same integrals: their
    ln I_i differ from the Gaussian unbinned ones by more than rounding and
    by less than one."""
    d = small_data
    base = L.lnl(d.o_events, d.o_cat, d.o_inj, LAM, T=8.6)["lnI"]
    for shape, nb in (("epanechnikov", 0), ("gaussian", 16)):
        r = L.lnl(d.o_events, d.o_cat, d.o_inj, LAM, T=8.6, shape=shape, n_bins=nb)["lnI"]
        diff = np.abs(r - base)
        print(shape, nb, diff.max())
        assert 1e-8 < diff.max() < 1.0


def test_bad_options_refused(small_data):
    d = small_data
    with pytest.raises(ValueError):
        L.lnl(d.o_events[:1], d.o_cat, d.o_inj, LAM, shape="box")
    with pytest.raises(ValueError):
        L.lnl(d.o_events[:1], d.o_cat, d.o_inj, LAM, n_bins=-1)
