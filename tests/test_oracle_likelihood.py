"""Pins of oracle.likelihood (no GPU): the bandwidth and KDE against scipy,
closed forms of the grid integral, invariances of ln L, the injection
estimator against its expectation."""
import copy
import math

import numpy as np
import pytest
from scipy import stats
from scipy.integrate import quad

from oracle import cosmology as C
from oracle import likelihood as L
from oracle.population import psi
from paper_2504_02034_amd import synth

LAM = synth.LAMBDA_TRUTH.copy()


def test_bandwidth_is_scipy_weighted_scott():
    rng = np.random.default_rng(7)
    z = rng.normal(0.8, 0.07, 3000)
    w = rng.gamma(2.0, 1e-3, 3000)
    kde = stats.gaussian_kde(z, weights=w)
    h = L.bandwidth(z, w, 1e-4)
    assert h == pytest.approx(math.sqrt(kde.covariance[0, 0]), rel=1e-12)


def test_kde_value_is_scipy():
    """n_r = delta at one node, g = 1: I = sum_j w_j N(z_k; z_j, h) = W1 kde(z_k)."""
    rng = np.random.default_rng(8)
    grid = np.linspace(0.0, 1.6, 1000)
    tau = L.trapezoid(grid)
    z = rng.normal(0.7, 0.05, 500)
    w = rng.gamma(2.0, 1e-3, 500)
    kde = stats.gaussian_kde(z, weights=w)
    for k in (380, 437, 470):
        nr = np.zeros(grid.size)
        nr[k] = 1.0 / tau[k]
        I, h = L.event_integral([z], [w], [1.0], [nr], grid, tau, np.ones(grid.size))
        assert I == pytest.approx(w.sum() * kde(grid[k])[0], rel=1e-12)


def test_grid_gaussian_normalised():
    """n = 1, g = 1, one sample: A = sum_g tau_g N(z_g; z_j, 2 dz) = 1 (h at its floor)."""
    grid = np.linspace(0.0, 1.6, 1000)
    tau = L.trapezoid(grid)
    for zj in (0.4, 0.40037, 1.1):
        I, h = L.event_integral([np.array([zj])], [np.array([1.0])], [1.0], [np.ones(1000)],
                                grid, tau, np.ones(1000))
        assert h == pytest.approx(2 * (grid[1] - grid[0]), rel=1e-15)
        assert I == pytest.approx(1.0, rel=1e-13)


def test_gaussian_convolution():
    """n(z) = N(z; zt, st), g = 1: A_j = N(z_j; zt, sqrt(h^2 + st^2))."""
    grid = np.linspace(0.0, 1.6, 4000)
    tau = L.trapezoid(grid)
    zt, st = 0.83, 0.004
    nr = stats.norm.pdf(grid, zt, st)
    d = 0.003
    z = np.array([0.83 - d, 0.83 + d])
    w = np.array([1.0, 1.0])
    I, h = L.event_integral([z], [w], [1.0], [nr], grid, tau, np.ones(grid.size))
    assert h == pytest.approx(math.sqrt(2) * d * 2 ** (-0.2), rel=1e-13)
    ref = np.sum(stats.norm.pdf(z, zt, math.hypot(h, st)))
    assert I == pytest.approx(ref, rel=1e-12)


def _run(d, lam=LAM, **kw):
    return L.lnl(d.o_events, d.o_cat, d.o_inj, lam, **kw)


def test_catalogue_scale_invariance(small_data):
    d = small_data
    base = _run(d)["lnl"]
    cat2 = L.Catalog(grid=d.o_cat.grid, rows={k: 3.7 * v for k, v in d.o_cat.rows.items()},
                     n_tot=3.7 * d.o_cat.n_tot)
    r = L.lnl(d.o_events, cat2, d.o_inj, LAM)
    assert r["lnl"] == pytest.approx(base, rel=1e-13)


def test_distance_scaling_identity(small_data):
    """d -> s d, H0 -> H0/s, p_draw -> p_draw/s  =>  ln L -> ln L - E ln s."""
    d = small_data
    s = 1.37
    base = _run(d)["lnl"]
    ev2 = copy.deepcopy(d.o_events)
    for e in ev2:
        for px in e.pixels:
            px.dl = px.dl * s
    inj2 = L.InjectionSet(d.o_inj.dl * s, d.o_inj.m1d, d.o_inj.m2d, d.o_inj.ln_pdraw - math.log(s),
                          d.o_inj.n_total)
    lam2 = LAM.copy(); lam2[0] /= s
    r = L.lnl(ev2, d.o_cat, inj2, lam2)
    assert r["lnl"] == pytest.approx(base - len(ev2) * math.log(s), rel=1e-12)


def test_permutations(small_data):
    d = small_data
    base = _run(d)
    rng = np.random.default_rng(9)
    order = rng.permutation(len(d.o_events))
    ev2 = [copy.deepcopy(d.o_events[i]) for i in order]
    for e in ev2:
        for px in e.pixels:
            p = rng.permutation(px.dl.size)
            px.dl, px.m1d, px.m2d = px.dl[p], px.m1d[p], px.m2d[p]
        e.pixels = [e.pixels[i] for i in rng.permutation(len(e.pixels))]
    r = L.lnl(ev2, d.o_cat, d.o_inj, LAM)
    assert r["lnl"] == pytest.approx(base["lnl"], rel=1e-13)
    assert np.allclose(r["lnI"], base["lnI"][order], rtol=1e-13)


def test_gr_independent_of_n(small_data):
    d = small_data
    a = LAM.copy(); a[3] = 0.5
    b = LAM.copy(); b[3] = 7.0
    assert _run(d, a)["lnl"] == _run(d, b)["lnl"]


def test_truncation_matches_dense(small_data):
    d = small_data
    assert _run(d, T=8.6)["lnl"] == pytest.approx(_run(d)["lnl"], rel=1e-14)


def test_domain_and_range(small_data):
    d = small_data
    bad = LAM.copy(); bad[7] = 4.0            # mmax < mmin
    assert _run(d, bad)["lnl"] == -np.inf
    far = LAM.copy(); far[0] = 1e6            # huge H0: distances beyond d(z=25)
    assert math.isnan(_run(d, far)["lnl"])
    empty = LAM.copy(); empty[6] = 200.0; empty[7] = 300.0; empty[8] = 250.0  # no sample in the support
    r = _run(d, empty)
    assert r["lnl"] == -np.inf and np.all(np.isneginf(r["lnI"]))
    nopeak = LAM.copy(); nopeak[8] = 500.0; nopeak[9] = 1.0  # peak has no mass in [mmin, mmax]
    assert _run(d, nopeak)["lnl"] == -np.inf


def test_selection_identical_injections():
    """All detected injections equal: xi = N_det s / N_inj, N_eff closed form."""
    grid = np.linspace(0, 1.6, 1000)
    cat = L.Catalog(grid=grid, rows={}, n_tot=np.ones(1000) / 1.6)
    nd, ni = 500, 20000
    inj = L.InjectionSet(np.full(nd, 3000.0), np.full(nd, 40.0), np.full(nd, 30.0),
                         np.full(nd, -12.0), ni)
    xi, neff, _ = L.selection(inj, cat, LAM)
    one = L.InjectionSet(inj.dl[:1], inj.m1d[:1], inj.m2d[:1], inj.ln_pdraw[:1], 1)
    s, _, _ = L.selection(one, cat, LAM)
    assert xi == pytest.approx(nd * s / ni, rel=1e-14)
    assert neff == pytest.approx(nd * nd / (nd - nd * nd / ni), rel=1e-12)


def test_selection_unbiased_for_all_detected():
    """With every proposal draw 'detected', xi estimates int p_pop(theta^d) dtheta^d
    = int n_tot(z) psi(z)/(1+z) dz (the masses integrate to one)."""
    rng = np.random.default_rng(10)
    n = 400_000
    dl = rng.uniform(1.0, 3e4, n)
    m1 = np.exp(rng.uniform(math.log(3.0), math.log(400.0), n))
    m2 = 3.0 + rng.random(n) * (m1 - 3.0)
    ln_p = -math.log(3e4 - 1) - np.log(m1) - math.log(math.log(400 / 3)) - np.log(m1 - 3.0)
    grid = np.linspace(0, 1.6, 1000)
    ntot = np.exp(-0.5 * ((grid - 0.8) / 0.3) ** 2)
    ntot /= np.sum(L.trapezoid(grid) * ntot)
    cat = L.Catalog(grid=grid, rows={}, n_tot=ntot)
    xi, neff, _ = L.selection(L.InjectionSet(dl, m1, m2, ln_p, n), cat, LAM)
    f = lambda z: np.interp(z, grid, ntot) * psi(z, LAM[11], LAM[12], LAM[13]) / (1 + z)
    ref = quad(f, 0, 1.6, limit=200)[0]
    assert xi == pytest.approx(ref, rel=5.0 / math.sqrt(neff))


def test_neff_gate(small_data):
    """The gate cuts exactly the points whose N_eff is at or below gate x N_ev."""
    d = small_data
    r = L.lnl(d.o_events, d.o_cat, d.o_inj, LAM)
    E = len(d.o_events)
    assert np.isfinite(r["lnl"]) and r["neff"] > 0
    just_below = r["neff"] / E * (1 - 1e-9)
    at = r["neff"] / E * (1 + 1e-12)
    assert L.lnl(d.o_events, d.o_cat, d.o_inj, LAM, neff_gate=just_below)["lnl"] == r["lnl"]
    assert L.lnl(d.o_events, d.o_cat, d.o_inj, LAM, neff_gate=at)["lnl"] == -np.inf
    assert L.lnl(d.o_events, d.o_cat, d.o_inj, LAM, neff_gate=0.0)["lnl"] == r["lnl"]
