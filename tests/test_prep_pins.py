"""Pins of the lambda-independent preparation that both sides consume.

* HEALPix RING geometry (Gorski et al. 2005), which both the oracle and the
  product take from the input generator: every pixel centre maps back to its
  own pixel; the nside = 1 centres are the twelve base-pixel centres; ring
  latitudes follow the cap / equatorial-belt formulas; the scheme is
  hierarchical (each nside-N pixel holds exactly four nside-2N centres) and
  equal-area (uniform points on the sphere fall into every pixel with equal
  probability).
* Sky factors (second factor of eq. gw-kernel-many1d): the pixel area times
  the 2-D KDE summed over the pixels around the event is the KDE's mass on
  the sphere, which the gnomonic projection fixes in closed form to second
  order in the angle.
* The product preparation equals the oracle's: the same regions and pixel
  ids, the same sky factors and the same catalogue rows.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2504_02034_amd import prep, synth


@pytest.mark.parametrize("nside", [1, 2, 32, 64])
def test_healpix_round_trip_every_pixel(nside):
    pix = np.arange(synth.nside_npix(nside))
    th, ph = synth.pix2ang_ring(nside, pix)
    assert np.array_equal(synth.ang2pix_ring(nside, th, ph), pix)


def test_healpix_base_pixel_centres():
    th, ph = synth.pix2ang_ring(1, np.arange(12))
    zc = np.cos(th)
    # four per zone: north cap at z = 2/3, the equator, south cap at z = -2/3
    assert np.allclose(zc, np.repeat([2.0 / 3.0, 0.0, -2.0 / 3.0], 4), atol=1e-15)
    q = math.pi / 4.0
    assert np.allclose(ph[:4], [q, 3 * q, 5 * q, 7 * q], atol=1e-15)
    assert np.allclose(ph[4:8], [0.0, 2 * q, 4 * q, 6 * q], atol=1e-15)
    assert np.allclose(ph[8:], [q, 3 * q, 5 * q, 7 * q], atol=1e-15)


@pytest.mark.parametrize("nside", [4, 64])
def test_healpix_rings(nside):
    """Ring i (1-based from the north pole) holds 4i pixels in the polar cap
    (i < N) and 4N in the belt, at z = 1 - i^2/(3N^2) and 4/3 - 2i/(3N)."""
    th, _ = synth.pix2ang_ring(nside, np.arange(synth.nside_npix(nside)))
    zs = np.cos(th)
    start = 0
    for i in range(1, 4 * nside):
        n_in = 4 * min(i, nside, 4 * nside - i)
        zr = zs[start:start + n_in]
        if i < nside:
            want = 1.0 - i * i / (3.0 * nside * nside)
        elif i <= 3 * nside:
            want = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
        else:
            j = 4 * nside - i
            want = -(1.0 - j * j / (3.0 * nside * nside))
        assert np.allclose(zr, want, atol=1e-14), i
        start += n_in
    assert start == synth.nside_npix(nside)


@pytest.mark.parametrize("nside", [1, 8, 32])
def test_healpix_hierarchy(nside):
    child = np.arange(synth.nside_npix(2 * nside))
    th, ph = synth.pix2ang_ring(2 * nside, child)
    parent = synth.ang2pix_ring(nside, th, ph)
    assert np.array_equal(np.bincount(parent, minlength=synth.nside_npix(nside)),
                          np.full(synth.nside_npix(nside), 4))


def test_healpix_equal_area():
    nside = 4
    npix = synth.nside_npix(nside)
    rng = np.random.default_rng(11)
    n = 2_000_000
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2 * math.pi, n)
    counts = np.bincount(synth.ang2pix_ring(nside, np.arccos(z), phi), minlength=npix)
    expect = n / npix
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    # chi-square with npix - 1 = 191 dof: mean 191, sd 19.5; 5 sd above the mean
    assert chi2 < 191 + 5 * 19.5, chi2


def _sky_sum_case(seed=3, n=800, sigma_deg=2.0):
    rng = np.random.default_rng(seed)
    th0, ph0 = 1.1, 2.3
    er = synth.unit_vectors(th0, ph0)
    ee = np.array([-math.sin(ph0), math.cos(ph0), 0.0])
    en = np.cross(er, ee)
    s = math.radians(sigma_deg)
    a, b = rng.normal(0, s, n), rng.normal(0, 0.6 * s, n)
    v = er[None, :] + a[:, None] * ee[None, :] + b[:, None] * en[None, :]
    th, ph = synth.vectors_to_angles(v)
    return th, ph


def _expected_sky_mass(th, ph):
    """The KDE is a density in the gnomonic plane, whose area element is
    d^2x = dOmega / cos^3(angle); to second order the mass on the sphere is
    1 - (3/2) E[|x|^2], with E[|x|^2] over the KDE = mean |x_j|^2 + trace of
    the kernel covariance."""
    v = synth.unit_vectors(th, ph)
    m = v.sum(axis=0)
    m /= np.linalg.norm(m)
    x = oracle.prep.tangent_plane(th, ph, m)
    cov = np.cov(x.T) * x.shape[0] ** (-1.0 / 3.0)
    return 1.0 - 1.5 * (np.mean(np.sum(x * x, axis=1)) + np.trace(cov)), m


@pytest.mark.parametrize("side", ["oracle", "product"])
def test_sky_factors_sum_to_the_kde_mass(side):
    th, ph = _sky_sum_case()
    want, m = _expected_sky_mass(th, ph)
    nside = 256
    pix_all = np.arange(synth.nside_npix(nside))
    ct, cp = synth.pix2ang_ring(nside, pix_all)
    near = synth.unit_vectors(ct, cp) @ m > math.cos(math.radians(12.0))
    area = synth.pixel_area(nside)
    if side == "oracle":
        s = oracle.prep.sky_factors(th, ph, ct[near], cp[near], area)
    else:
        s = prep._sky_factors(th, ph, ct[near], cp[near], area)
    total = float(np.sum(s))
    # the midpoint rule on pixels of 0.23 deg is exact to ~1e-10 against a
    # kernel of ~0.6 deg; what is left is the fourth order of the projection
    # (1.4e-5 here).  A wrong bandwidth exponent moves the sum by ~1e-3.
    assert abs(total - want) < 5e-5, (total, want)
    assert 0.99 < total < 1.0


def test_product_prep_equals_oracle_prep(small_data):
    d = small_data
    p = d.prep
    assert p.n_events == len(d.o_events)
    for e, oe in enumerate(d.o_events):
        qs = range(p.ev_pix_off[e], p.ev_pix_off[e + 1])
        assert [int(p.pix_id[q]) for q in qs] == [px.pix for px in oe.pixels]
        for q, px in zip(qs, oe.pixels):
            sl = slice(p.pix_samp_off[q], p.pix_samp_off[q + 1])
            assert np.array_equal(np.sort(p.dl[sl]), np.sort(px.dl))
            assert abs(p.c_ir[q] - px.c) <= 1e-14 * abs(px.c)
    for i, pid in enumerate(p.row_pix):
        o_row = d.o_cat.rows[int(pid)]
        scale = max(float(np.max(np.abs(o_row))), 1e-300)
        assert np.max(np.abs(p.nz[i] - o_row)) <= 1e-13 * scale, int(pid)
    tot_scale = float(np.max(np.abs(d.o_cat.n_tot)))
    assert np.max(np.abs(p.nz_tot - d.o_cat.n_tot)) <= 1e-13 * tot_scale
