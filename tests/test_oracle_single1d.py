"""Pins of the oracle's single-1D kernel (eq. gw-kernel-single1d, Sect. 2.3),
no GPU: a Gaussian-convolution closed form on two pixels whose samples and
weights differ, the reduction to the many-1D kernel when every pixel of an
event holds the same samples, the invariance under moving a sample to
another pixel with the pixel's sky factor kept, and the samples outside the
region entering the KDE (the 30-digit brute force of both kernels, with
out-of-region samples, is in test_oracle_bruteforce.py)."""
import copy
import math

import numpy as np
import pytest
from scipy import stats

from oracle import likelihood as L
from paper_2504_02034_amd import synth

LAM = synth.LAMBDA_TRUTH.copy()


def _two_pixel_case():
    grid = np.linspace(0.0, 1.6, 4000)
    tau = L.trapezoid(grid)
    st = 0.004
    zt = (0.80, 0.86)
    rows = [stats.norm.pdf(grid, m, st) for m in zt]
    z = [np.array([0.825]), np.array([0.829, 0.834])]
    w = [np.array([2.0]), np.array([0.5, 1.5])]
    c = [0.7, 0.2]
    return grid, tau, st, zt, rows, z, w, c


def test_two_pixel_gaussian_convolution():
    """n_r = N(z; zt_r, st), g = 1: the grid integral of N(z; z_j, h) n_r is
    N(z_j; zt_r, sqrt(h^2 + st^2)), so
    I = sum_r c_r N_r (1/N) sum_{all j} w_j N(z_j; zt_r, sqrt(h^2 + st^2)),
    which differs from the many-1D sum over each pixel's own samples."""
    grid, tau, st, zt, rows, z, w, c = _two_pixel_case()
    z_all, w_all = np.concatenate(z), np.concatenate(w)
    s_ir = [c[r] * z[r].size for r in range(2)]
    I, h = L.event_integral_single1d(z_all, w_all, s_ir, rows, grid, tau, np.ones(grid.size))
    assert h == pytest.approx(L.bandwidth(z_all, w_all, grid[1] - grid[0]), rel=0)
    s = math.hypot(h, st)
    ref = sum(c[r] * z[r].size * np.sum(w_all * stats.norm.pdf(z_all, zt[r], s)) / z_all.size
              for r in range(2))
    assert I == pytest.approx(ref, rel=1e-12)
    many = sum(c[r] * np.sum(w[r] * stats.norm.pdf(z[r], zt[r], s)) for r in range(2))
    I_many, _ = L.event_integral(z, w, c, rows, grid, tau, np.ones(grid.size))
    assert I_many == pytest.approx(many, rel=1e-12)
    assert abs(I - I_many) > 0.05 * I


@pytest.fixture(scope="module")
def small_data():
    from tests.datasets import small
    return small()


def _same_samples_everywhere(events):
    """Every pixel of each event takes the event's first pixel's samples, and
    the event holds no samples outside its pixels; sky factors S = c N."""
    out = copy.deepcopy(events)
    for e in out:
        p0 = e.pixels[0]
        for px in e.pixels[1:]:
            px.dl, px.m1d, px.m2d = p0.dl.copy(), p0.m1d.copy(), p0.m2d.copy()
        for px in e.pixels:
            px.s = None
        e.samples = None
    return out


@pytest.mark.parametrize("T", [None, 8.6])
def test_identical_pixels_reduce_to_many1d(small_data, T):
    """With the same R-sample multiset in every pixel and none outside, the
    event KDE is each pixel's KDE and S_ir = c_ir N_r, so both kernels give
    the same I_i."""
    d = small_data
    ev = _same_samples_everywhere(d.o_events[:4])
    assert any(len(e.pixels) > 1 for e in ev)
    a = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=T, kernel="single1d")
    b = L.lnl(ev, d.o_cat, d.o_inj, LAM, T=T, kernel="many1d")
    assert np.all(np.isfinite(a["lnI"]))
    assert np.allclose(a["lnI"], b["lnI"], rtol=1e-13, atol=0)
    assert np.array_equal(a["h"], b["h"])


def test_moving_a_sample_keeps_single1d(small_data):
    """The single-1D KDE does not see which pixel holds a sample: moving one
    sample from pixel 0 to pixel 1, with the sky factors kept, leaves I_i
    unchanged, while the many-1D value changes."""
    d = small_data
    e = next(copy.deepcopy(e) for e in d.o_events if len(e.pixels) > 1
             and e.pixels[0].dl.size > 1)
    e.samples = None
    for px in e.pixels:
        px.s = None
    ref = L.lnl([e], d.o_cat, d.o_inj, LAM, T=8.6, kernel="single1d")["lnI"][0]
    ref_many = L.lnl([e], d.o_cat, d.o_inj, LAM, T=8.6, kernel="many1d")["lnI"][0]
    p0, p1 = e.pixels[0], e.pixels[1]
    s0, s1 = p0.c * p0.dl.size, p1.c * p1.dl.size
    for a in ("dl", "m1d", "m2d"):
        setattr(p1, a, np.append(getattr(p1, a), getattr(p0, a)[-1]))
        setattr(p0, a, getattr(p0, a)[:-1])
    p0.c, p1.c = s0 / p0.dl.size, s1 / p1.dl.size
    got = L.lnl([e], d.o_cat, d.o_inj, LAM, T=8.6, kernel="single1d")["lnI"][0]
    got_many = L.lnl([e], d.o_cat, d.o_inj, LAM, T=8.6, kernel="many1d")["lnI"][0]
    assert got == pytest.approx(ref, rel=1e-13, abs=0)
    assert abs(got_many - ref_many) > 1e-6


def test_samples_outside_the_pixels_enter_the_kde(small_data):
    """The single-1D KDE is trained on all N_i samples of the event: with the
    out-of-region samples it equals the closed sum written out here over the
    whole sample list, and differs from the value over the pixels' samples."""
    d = small_data
    e = next(e for e in d.o_events
             if e.samples[0].size > sum(px.dl.size for px in e.pixels))
    full = L.lnl([e], d.o_cat, d.o_inj, LAM, kernel="single1d")
    inner = copy.deepcopy(e)
    inner.samples = None
    part = L.lnl([inner], d.o_cat, d.o_inj, LAM, kernel="single1d")
    assert abs(full["lnI"][0] - part["lnI"][0]) > 1e-6
    z, w = L.redshift_and_weight(*e.samples, LAM)
    grid = d.o_cat.grid
    h = L.bandwidth(z, w, grid[1] - grid[0])
    kde = np.array([np.sum(w * stats.norm.pdf(zg, z, h)) for zg in grid]) / z.size
    tau, gz = L.trapezoid(grid), L.grid_factor(grid, LAM)
    I = sum(px.s * np.sum(tau * d.o_cat.rows[px.pix] * gz * kde) for px in e.pixels)
    assert full["h"][0] == pytest.approx(h, rel=1e-14)
    assert full["lnI"][0] == pytest.approx(math.log(I), rel=1e-13)


def test_unknown_kernel_refused(small_data):
    d = small_data
    with pytest.raises(ValueError):
        L.lnl(d.o_events[:1], d.o_cat, d.o_inj, LAM, kernel="two1d")
