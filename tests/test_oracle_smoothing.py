"""Pins of the oracle's smoothed lower mass edge (Table 1's delta_m), no GPU:
the smoothing function's closed values, both smoothed densities integrating
to 1 over their supports (scipy quad, independent of the normalisations the
oracle computes), delta_m = 0 giving the unsmoothed model bitwise, and the
weight through ln L."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import likelihood as L
from oracle import population as pop
from paper_2504_02034_amd import synth

LAM15 = np.append(synth.LAMBDA_TRUTH, 4.8)      # the paper's fiducial delta_m


def test_smoothing_closed_values():
    mmin, dm = 5.0, 4.8
    assert float(pop.smoothing(mmin, mmin, dm)) == 0.0
    assert float(pop.smoothing(mmin - 1.0, mmin, dm)) == 0.0
    assert float(pop.smoothing(mmin + dm, mmin, dm)) == 1.0
    assert float(pop.smoothing(mmin + 0.5 * dm, mmin, dm)) == pytest.approx(0.5, abs=1e-15)
    m = np.linspace(mmin, mmin + dm, 1001)
    s = pop.smoothing(m, mmin, dm)
    assert np.all(np.diff(s) >= 0.0)
    # S(mmin + x) + S(mmin + dm - x) = 1 (the exponent changes sign)
    x = np.linspace(0.01, dm - 0.01, 37)
    assert np.allclose(pop.smoothing(mmin + x, mmin, dm) + pop.smoothing(mmin + dm - x, mmin, dm),
                       1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dm", [4.8, 0.7, 95.0])
def test_smoothed_densities_integrate_to_one(dm):
    lam = LAM15.copy()
    lam[14] = dm
    mmin, mmax = lam[6], lam[7]
    pts = [mmin + dm] if mmin + dm < mmax else None

    def p1(m):        # marginal of m1: integrate w over m2 in [mmin, m1]
        return quad(lambda m2: float(pop.mass_weight(np.array([m]), np.array([m2]), lam)[0]),
                    mmin, m, epsabs=0, epsrel=1e-11, limit=200)[0]

    for m1 in (mmin + 0.3 * min(dm, mmax - mmin), 40.0, 80.0):
        if m1 <= mmin or m1 > mmax:
            continue
        got = p1(m1)
        n1, q = pop.smoothed_constants(lam)
        direct = float(pop.p_m1(m1, *lam[[4, 6, 7, 8, 9, 10]]) * pop.smoothing(m1, mmin, dm)) / n1
        assert got == pytest.approx(direct, rel=1e-9)     # p(m2|m1) integrates to 1
    tot = quad(lambda m: float(pop.p_m1(m, *lam[[4, 6, 7, 8, 9, 10]])
                               * pop.smoothing(m, mmin, dm)), mmin, mmax,
               points=pts, epsabs=0, epsrel=1e-12, limit=400)[0]
    assert tot / pop.smoothed_constants(lam)[0] == pytest.approx(1.0, rel=1e-10)


def test_zero_delta_m_is_the_unsmoothed_model():
    rng = np.random.default_rng(2)
    m1 = rng.uniform(3.0, 95.0, 500)
    m2 = m1 * rng.uniform(0.2, 1.0, 500)
    lam14 = synth.LAMBDA_TRUTH.copy()
    lam15 = np.append(lam14, 0.0)
    assert np.array_equal(pop.mass_weight(m1, m2, lam14), pop.mass_weight(m1, m2, lam15))
    w_s = pop.mass_weight(m1, m2, LAM15)
    w_u = pop.mass_weight(m1, m2, lam14)
    far = (m2 > lam14[6] + 4.8) & (m1 > lam14[6] + 4.8)
    # away from the edge the smoothed weight is the unsmoothed one times the
    # two normalisation ratios, the same for every sample with the same m1 regime
    r = w_s[far & (w_u > 0)] / w_u[far & (w_u > 0)]
    assert r.size > 10 and np.all(r > 0)


def test_through_ln_l():
    from tests.datasets import small
    d = small()
    a = L.lnl(d.o_events[:2], d.o_cat, d.o_inj, LAM15, T=8.6)
    b = L.lnl(d.o_events[:2], d.o_cat, d.o_inj, synth.LAMBDA_TRUTH, T=8.6)
    assert np.isfinite(a["lnl"]) and a["lnl"] != b["lnl"]
    bad = LAM15.copy()
    bad[14] = -1.0
    assert L.lnl(d.o_events[:2], d.o_cat, d.o_inj, bad)["lnl"] == -np.inf
