"""Pins of the oracle gradient (oracle/gradient.py): every piece against
Richardson central differences of the oracle function it differentiates,
the whole d ln L / d lambda against differences of likelihood.lnl on small
inputs, and the exact zeros of the modified-propagation derivatives at
their GR points (eq. dL-mg: Xi = 1 at Xi0 = 1 for every n, and at n = 0 for
every Xi0)."""
import numpy as np
import pytest

import oracle
from oracle import cosmology as cosmo
from oracle import gradient as G
from oracle import likelihood as L
from paper_2504_02034_amd import synth
from tests.datasets import handcrafted, handcrafted_oracle

TRUTH = synth.LAMBDA_TRUTH
OTHER = np.array([88.0, 0.41, 1.7, 3.2, 2.6, 0.7, 5.0, 87.0, 31.0, 4.4, 0.3, 2.1, 2.4, 1.6])


def rel_close(a, b, tol, floor=1.0):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.all(np.abs(a - b) <= tol * np.maximum(floor, np.abs(b)))


@pytest.mark.parametrize("om", [0.1, 0.3, 0.93])
def test_dchi_dom(om):
    z = np.array([0.05, 0.4, 1.3, 4.0, 17.0])
    fd = G.richardson(lambda l: cosmo.chi(z, l[1]), np.array([70.0, om, 1, 0]), 1)
    assert rel_close(G.dchi_dom(z, om), fd, 1e-9, floor=1e-12)


@pytest.mark.parametrize("lam", [TRUTH, OTHER])
def test_distance_parts(lam):
    z = np.array([0.02, 0.3, 0.9, 1.6, 6.0])
    D, Dz, Dzz, dD, dDz = G.distance_parts(z, lam)
    assert rel_close(D, cosmo.dl_gw(z, *lam[:4]), 1e-14)
    assert rel_close(Dz, cosmo.ddl_gw_dz(z, *lam[:4]), 1e-14)
    # d2D/dz2: differences of dD/dz in z (z shifted by s - 1 around s = 1)
    fz = G.richardson(lambda s: cosmo.ddl_gw_dz(z + (s[0] - 1.0), *lam[:4]), np.array([1.0]), 0,
                      rel_step=1e-4)
    assert rel_close(Dzz, fz, 1e-8)
    for p in range(4):
        fd = G.richardson(lambda l: cosmo.dl_gw(z, *l[:4]), lam, p)
        fdz = G.richardson(lambda l: cosmo.ddl_gw_dz(z, *l[:4]), lam, p)
        assert rel_close(dD[p], fd, 1e-8, floor=1e-6 * np.abs(D).max()), p
        assert rel_close(dDz[p], fdz, 1e-8, floor=1e-6 * np.abs(Dz).max()), p


def test_redshift_derivative_is_the_inverse_function_derivative():
    d = np.array([300.0, 2500.0, 9000.0, 21000.0])
    for lam in (TRUTH, OTHER):
        z = cosmo.invert_dl(d, *lam[:4])
        dz = G.dz_dparams(z, lam)
        for p in range(4):
            fd = G.richardson(lambda l: cosmo.invert_dl(d, *l[:4]), lam, p)
            assert rel_close(dz[p], fd, 1e-7, floor=1e-9), p
        assert np.all(dz[4:] == 0.0)


@pytest.mark.parametrize("lam", [TRUTH, OTHER])
def test_mass_log_derivatives(lam):
    rng = np.random.default_rng(3)
    m1 = rng.uniform(8.0, 80.0, 40)
    m2 = m1 * rng.uniform(0.3, 0.98, 40)
    m2 = np.maximum(m2, 5.5)
    d, mdm = G.mass_log_derivs(m1, m2, lam)
    lw = lambda l: np.log(oracle.population.mass_weight(m1, m2, l))  # noqa: E731
    for k, p in enumerate((4, 5, 8, 9, 10)):
        fd = G.richardson(lw, lam, p, rel_step=1e-4, abs_floor=1e-5)
        assert rel_close(d[k], fd, 2e-7, floor=1e-4), p
    # m1 dlnw/dm1 + m2 dlnw/dm2 = d ln w(s m1, s m2) / d ln s at s = 1
    fs = G.richardson(lambda s: np.log(oracle.population.mass_weight(m1 * s[0], m2 * s[0], lam)),
                      np.array([1.0]), 0, rel_step=1e-5)
    assert rel_close(mdm, fs, 2e-7)


def test_mass_log_derivatives_at_special_forms():
    m1 = np.array([12.0, 40.0, 70.0])
    m2 = np.array([9.0, 20.0, 50.0])
    for a, b in ((1.0, 1.1), (3.4, -1.0)):
        lam = TRUTH.copy()
        lam[4], lam[5] = a, b
        d, _ = G.mass_log_derivs(m1, m2, lam)
        lw = lambda l: np.log(oracle.population.mass_weight(m1, m2, l))  # noqa: E731
        for k, p in enumerate((4, 5)):
            fd = G.richardson(lw, lam, p, rel_step=1e-4)
            assert rel_close(d[k], fd, 1e-6, floor=1e-6), (a, b, p)


def test_psi_log_derivatives():
    z = np.array([0.0, 0.4, 1.2, 3.0])
    for lam in (TRUTH, OTHER):
        d, dz = G.psi_log_derivs(z, lam)
        lp = lambda l: np.log(oracle.population.psi(z, l[11], l[12], l[13]))  # noqa: E731
        for k, p in enumerate((11, 12, 13)):
            assert rel_close(d[k], G.richardson(lp, lam, p), 1e-8, floor=1e-8)
        fz = G.richardson(lambda s: np.log(oracle.population.psi(z + s[0] - 1.0, *lam[11:])),
                          np.array([1.0]), 0)
        assert rel_close(dz, fz, 1e-8, floor=1e-8)


@pytest.fixture(scope="module")
def hand():
    h = handcrafted()
    return h, handcrafted_oracle(h)


def _lnl(structs, T, kernel="many1d"):
    events, cat, inj = structs
    return lambda l: L.lnl(events, cat, inj, l, T=T, kernel=kernel)["lnl"]


def _xi(structs):
    events, cat, inj = structs
    return lambda l: np.log(L.selection(inj, cat, l)[0])


@pytest.mark.parametrize("lam", [TRUTH, OTHER], ids=["truth", "other"])
def test_selection_gradient_vs_differences(hand, lam):
    _, structs = hand
    events, cat, inj = structs
    xi, dlnxi = G.selection_grad(inj, cat, lam)
    assert xi == pytest.approx(L.selection(inj, cat, lam)[0], rel=1e-14)
    f = _xi(structs)
    for k, p in enumerate(G.GRAD_INDEX):
        fd = G.richardson(f, lam, p, rel_step=1e-6)
        assert abs(dlnxi[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, dlnxi[k], fd)


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
@pytest.mark.parametrize("T", [None, 8.6], ids=["dense", "T8.6"])
@pytest.mark.parametrize("lam", [TRUTH, OTHER], ids=["truth", "other"])
def test_lnl_gradient_vs_differences(hand, lam, T, kernel):
    _, structs = hand
    events, cat, inj = structs
    res = G.lnl_grad(events, cat, inj, lam, T=T, kernel=kernel)
    ref = L.lnl(events, cat, inj, lam, T=T, kernel=kernel)
    assert res["lnl"] == pytest.approx(ref["lnl"], rel=1e-13)
    assert np.allclose(res["lnI"], ref["lnI"], rtol=1e-13, atol=0)
    f = _lnl(structs, T, kernel)
    for k, p in enumerate(G.GRAD_INDEX):
        fd = G.richardson(f, lam, p, rel_step=1e-6)
        assert abs(res["grad"][k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, res["grad"][k], fd)


def test_modified_propagation_derivatives_vanish_at_gr(hand):
    _, (events, cat, inj) = hand
    gr = OTHER.copy()
    gr[2] = 1.0
    g = G.lnl_grad(events, cat, inj, gr)["grad"]
    assert g[3] == 0.0 and np.all(np.isfinite(g))
    n0 = OTHER.copy()
    n0[3] = 0.0
    g = G.lnl_grad(events, cat, inj, n0)["grad"]
    assert g[2] == 0.0 and np.all(np.isfinite(g))


def test_gradient_nan_outside_domain(hand):
    _, (events, cat, inj) = hand
    bad = TRUTH.copy()
    bad[1] = 1.5
    r = G.lnl_grad(events, cat, inj, bad)
    assert r["lnl"] == -np.inf and np.all(np.isnan(r["grad"]))


# ---------------------------------------------------------------------------
# incomplete catalogue (eqs. p-gal, p-miss, f-R): the rows and n_tot depend on
# Om through the completion density and f_R
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("om", [0.12, 0.3, 0.8])
def test_completion_density_dom(om):
    z = np.array([0.0, 0.02, 0.4, 1.1, 1.6])
    an = G.completion_density_dom(z, om, 1.6)
    for i, zz in enumerate(z):
        fd = G.richardson(lambda l: float(L.completion_density(np.array([zz]), l[1], 1.6)[0]),
                          np.array([70.0, om]), 1)
        assert abs(an[i] - fd) <= 1e-8 * max(1e-3, abs(fd)), (zz, an[i], fd)


@pytest.fixture(scope="module")
def hand_incomplete(hand):
    """The handcrafted structures with a smooth per-row completeness and M(z)."""
    import copy
    _, (events, cat, inj) = hand
    grid = cat.grid
    c = copy.copy(cat)
    c.p_compl = {r: 1.0 / (1.0 + np.exp((grid - (0.5 + 0.15 * r)) / 0.1)) for r in cat.rows}
    c.missing = 4.0 * np.pi * (0.2 + 0.6 / (1.0 + np.exp(-(grid - 0.8) / 0.2)))
    return events, c, inj


@pytest.mark.parametrize("lam", [TRUTH, OTHER], ids=["truth", "other"])
def test_selection_gradient_with_incompleteness(hand_incomplete, lam):
    events, cat, inj = hand_incomplete
    xi, dlnxi = G.selection_grad(inj, cat, lam)
    assert xi == pytest.approx(L.selection(inj, cat, lam)[0], rel=1e-14)
    f = _xi(hand_incomplete)
    for k, p in enumerate(G.GRAD_INDEX):
        fd = G.richardson(f, lam, p, rel_step=1e-6)
        assert abs(dlnxi[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, dlnxi[k], fd)


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
@pytest.mark.parametrize("lam", [TRUTH, OTHER], ids=["truth", "other"])
def test_lnl_gradient_with_incompleteness(hand_incomplete, lam, kernel):
    events, cat, inj = hand_incomplete
    res = G.lnl_grad(events, cat, inj, lam, T=8.6, kernel=kernel)
    ref = L.lnl(events, cat, inj, lam, T=8.6, kernel=kernel)
    assert res["lnl"] == pytest.approx(ref["lnl"], rel=1e-13)
    f = _lnl(hand_incomplete, 8.6, kernel)
    for k, p in enumerate(G.GRAD_INDEX):
        fd = G.richardson(f, lam, p, rel_step=1e-6)
        assert abs(res["grad"][k] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, res["grad"][k], fd)
    # the incompleteness moves d ln L / d Om
    plain = G.lnl_grad(events, hand_incomplete_plain(cat), inj, lam, T=8.6, kernel=kernel)
    assert abs(plain["grad"][1] - res["grad"][1]) > 1e-3


def hand_incomplete_plain(cat):
    import copy
    c = copy.copy(cat)
    c.p_compl = None
    c.missing = None
    return c


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
@pytest.mark.parametrize("lam", [TRUTH, OTHER], ids=["truth", "other"])
def test_epanechnikov_gradient_vs_differences(hand, lam, kernel):
    """The compact kernel of Sect. 2.3 (the Epanechnikov option): the
    analytic gradient against Richardson differences of likelihood.lnl with
    the same kernel.  dk/dh and dk/dz_j do not vanish at the support's edge,
    so ln L has a kink wherever a grid point crosses an edge: a difference
    whose steps straddle one is off (event 2 at OTHER, H0: 7e-5 at 1e-6,
    4e-10 at 1e-7).  Each parameter is also differenced at a step ten times
    smaller, and one of the two must agree."""
    _, structs = hand
    events, cat, inj = structs
    res = G.lnl_grad(events, cat, inj, lam, kernel=kernel, shape="epanechnikov")
    ref = L.lnl(events, cat, inj, lam, kernel=kernel, shape="epanechnikov")
    assert np.isfinite(ref["lnl"])
    assert res["lnl"] == pytest.approx(ref["lnl"], rel=1e-13)
    assert np.allclose(res["lnI"], ref["lnI"], rtol=1e-13, atol=0)
    f = lambda l: L.lnl(events, cat, inj, l, kernel=kernel, shape="epanechnikov")["lnl"]  # noqa: E731
    for k, p in enumerate(G.GRAD_INDEX):
        fds = [G.richardson(f, lam, p, rel_step=st, abs_floor=st) for st in (1e-6, 1e-7)]
        err = min(abs(res["grad"][k] - fd) / max(1.0, abs(fd)) for fd in fds)
        assert err <= 1e-6, (k, res["grad"][k], fds)


def test_epanechnikov_gradient_differs_from_the_gaussian(hand):
    """The shape reaches the gradient (a plausible slip would ignore it)."""
    _, (events, cat, inj) = hand
    g = G.lnl_grad(events, cat, inj, TRUTH)["grad"]
    e = G.lnl_grad(events, cat, inj, TRUTH, shape="epanechnikov")["grad"]
    assert np.all(np.isfinite(e)) and np.max(np.abs(e - g)) > 1e-3 * np.max(np.abs(g))


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
def test_epanechnikov_gradient_with_incompleteness(hand_incomplete, kernel):
    """The compact kernel with an incomplete catalogue: the rows' own Om
    dependence weighted by the polynomial kernel (differences at two steps,
    as above)."""
    events, cat, inj = hand_incomplete
    lam = OTHER
    res = G.lnl_grad(events, cat, inj, lam, kernel=kernel, shape="epanechnikov")
    ref = L.lnl(events, cat, inj, lam, kernel=kernel, shape="epanechnikov")
    assert np.isfinite(ref["lnl"]) and res["lnl"] == pytest.approx(ref["lnl"], rel=1e-13)
    f = lambda l: L.lnl(events, cat, inj, l, kernel=kernel, shape="epanechnikov")["lnl"]  # noqa: E731
    for k, p in enumerate(G.GRAD_INDEX):
        fds = [G.richardson(f, lam, p, rel_step=st, abs_floor=st) for st in (1e-6, 1e-7)]
        err = min(abs(res["grad"][k] - fd) / max(1.0, abs(fd)) for fd in fds)
        assert err <= 1e-6, (k, res["grad"][k], fds)


@pytest.mark.parametrize("kernel,shape,n_bins", [("many1d", "gaussian", 4),
                                                 ("single1d", "gaussian", 8),
                                                 ("many1d", "epanechnikov", 4)])
def test_binned_gradient_vs_differences(hand, kernel, shape, n_bins):
    """Binned data sets (Sect. 2.3): the bins' centres move with the ends of
    the redshift range and their weights with the samples' weights; ln L
    jumps when a sample changes bins, so each parameter is differenced at two
    steps and one must agree."""
    _, structs = hand
    events, cat, inj = structs
    lam = OTHER
    T = 8.6 if shape == "gaussian" else None
    res = G.lnl_grad(events, cat, inj, lam, T=T, kernel=kernel, shape=shape, n_bins=n_bins)
    ref = L.lnl(events, cat, inj, lam, T=T, kernel=kernel, shape=shape, n_bins=n_bins)
    assert np.isfinite(ref["lnl"]) and res["lnl"] == pytest.approx(ref["lnl"], rel=1e-13)
    f = lambda l: L.lnl(events, cat, inj, l, T=T, kernel=kernel, shape=shape,  # noqa: E731
                        n_bins=n_bins)["lnl"]
    for k, p in enumerate(G.GRAD_INDEX):
        fds = [G.richardson(f, lam, p, rel_step=st, abs_floor=st) for st in (1e-6, 1e-7)]
        err = min(abs(res["grad"][k] - fd) / max(1.0, abs(fd)) for fd in fds)
        assert err <= 1e-6, (k, res["grad"][k], fds)
    plain = G.lnl_grad(events, cat, inj, lam, T=T, kernel=kernel, shape=shape)
    assert np.max(np.abs(plain["grad"] - res["grad"])) > 1e-6
