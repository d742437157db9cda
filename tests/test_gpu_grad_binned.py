"""The adjoint on binned data sets (Sect. 2.3) through chimera_lnl_grad
against the oracle's gradient (oracle.gradient.lnl_grad with n_bins): the
10-event data, many-1D and single-1D, Gaussian and Epanechnikov kernels,
FP64 at 1e-8 per component (relative to max(1, |g|)), ln L equal to the
forward call's, FP32 against FP64; the unbinned gradient back once the set
is reset."""
import numpy as np
import pytest

from paper_2504_02034_amd import synth

pytestmark = pytest.mark.gpu
SHAPES = {"gaussian": 0, "epanechnikov": 1}


def rel_err(got, ref):
    return np.abs(got - ref) / np.maximum(1.0, np.abs(ref))


@pytest.fixture(scope="module")
def small(small_data):
    from paper_2504_02034_amd import chimera, prep
    d = small_data
    ctx, many = chimera.context_from_prepared(d.prep, d.inj)
    sets = {"many1d": many, "single1d": ctx.add_prepared_single1d(prep.single1d(d.prep, d.ev))}
    rng = np.random.default_rng(9)
    lam = np.stack([synth.LAMBDA_TRUTH] +
                   [synth.LAMBDA_TRUTH * (1.0 + rng.uniform(-0.05, 0.05, 14)) for _ in range(3)])
    yield d, chimera, ctx, sets, lam
    ctx.close()


@pytest.mark.parametrize("kernel,shape,n_bins", [("many1d", "gaussian", 16),
                                                 ("single1d", "gaussian", 64),
                                                 ("many1d", "epanechnikov", 16),
                                                 ("many1d", "gaussian", 1)])
def test_binned_gradient_matches_oracle(small, kernel, shape, n_bins):
    from oracle import gradient as G
    d, chimera, ctx, sets, lam = small
    ev = sets[kernel]
    _, g_plain = ctx.lnl_grad(ev, lam, chimera.CHIMERA_FP64)
    ctx.set_event_kde(ev, SHAPES[shape], n_bins)
    try:
        lnl, grad = ctx.lnl_grad(ev, lam, chimera.CHIMERA_FP64)
        lnl_f = ctx.lnl(ev, lam, chimera.CHIMERA_FP64)
        _, g32 = ctx.lnl_grad(ev, lam, chimera.CHIMERA_FP32)
    finally:
        ctx.set_event_kde(ev)
    _, g_back = ctx.lnl_grad(ev, lam, chimera.CHIMERA_FP64)
    assert np.array_equal(g_back, g_plain, equal_nan=True)
    fin = np.isfinite(lnl)
    assert fin.sum() >= 3 and np.array_equal(np.isfinite(lnl_f), fin)
    assert np.all(np.abs(lnl[fin] - lnl_f[fin]) <= 1e-11 * np.abs(lnl_f[fin]))
    T = 8.6 if shape == "gaussian" else None
    for b in range(lam.shape[0]):
        ref = G.lnl_grad(d.o_events, d.o_cat, d.o_inj, lam[b], T=T, kernel=kernel, shape=shape,
                         n_bins=n_bins)
        if not np.isfinite(ref["lnl"]):
            assert not np.isfinite(lnl[b])
            continue
        assert abs(lnl[b] - ref["lnl"]) <= 1e-10 * max(1.0, abs(ref["lnl"])), (b, lnl[b])
        err = rel_err(grad[b], ref["grad"])
        assert np.all(err <= 1e-8), (b, err)
    assert np.max(np.abs(grad[fin] - g_plain[fin])) > 1e-6      # the bins reach the gradient
    e32 = rel_err(g32[fin], grad[fin])
    print(kernel, shape, n_bins, "FP32 vs FP64", e32.max())
    assert e32.max() <= 1e-2


@pytest.mark.parametrize("kernel,shape", [("many1d", "gaussian"), ("single1d", "epanechnikov")])
def test_binned_gradient_with_incomplete_catalogue(small, kernel, shape):
    """Binned sets with an incomplete catalogue: the completed rows and their
    Om derivative under the bins (16 per data set), against the oracle at
    1e-8."""
    import copy
    from oracle import gradient as G
    d, chimera, ctx, sets, lam = small
    ev = sets[kernel]
    p_rows, missing = synth.make_completeness(d.prep.row_pix, d.wl.nside, d.grid)
    o_cat = copy.copy(d.o_cat)
    o_cat.p_compl = {int(px): p_rows[i] for i, px in enumerate(d.prep.row_pix)}
    o_cat.missing = missing
    ctx.set_completeness(p_rows, missing)
    ctx.set_event_kde(ev, SHAPES[shape], 16)
    try:
        lnl, grad = ctx.lnl_grad(ev, lam, chimera.CHIMERA_FP64)
        lnl_f = ctx.lnl(ev, lam, chimera.CHIMERA_FP64)
    finally:
        ctx.set_event_kde(ev)
        ctx.set_completeness(None)
    fin = np.isfinite(lnl)
    assert fin.sum() >= 3 and np.array_equal(np.isfinite(lnl_f), fin)
    T = 8.6 if shape == "gaussian" else None
    for b in range(lam.shape[0]):
        ref = G.lnl_grad(d.o_events, o_cat, d.o_inj, lam[b], T=T, kernel=kernel, shape=shape,
                         n_bins=16)
        if not np.isfinite(ref["lnl"]):
            assert not np.isfinite(lnl[b])
            continue
        assert abs(lnl[b] - ref["lnl"]) <= 1e-10 * max(1.0, abs(ref["lnl"])), (b, lnl[b])
        err = rel_err(grad[b], ref["grad"])
        assert np.all(err <= 1e-8), (b, err)
