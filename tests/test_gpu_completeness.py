"""An incomplete catalogue (eqs. p-gal, p-miss, f-R) through the C-ABI
(chimera_set_completeness) against the oracle: ln I_i, ln xi and ln L at
1e-10 (FP64) for the many-1D, single-1D, Epanechnikov and 3D kernels with a
synthetic per-pixel completeness, FP32 within 1e-3, the adjoint against the
oracle's gradient, the complete catalogue back bitwise once it is cleared,
and the values the call refuses."""
import copy
import math

import numpy as np
import pytest

from paper_2504_02034_amd import synth

pytestmark = pytest.mark.gpu
REL64 = 1e-10


def close(a, b, rel):
    if math.isnan(b):
        return math.isnan(a)
    if math.isinf(b):
        return a == b
    return abs(a - b) <= rel * max(1.0, abs(b))


@pytest.fixture(scope="module")
def setup(small_data):
    from paper_2504_02034_amd import chimera, prep
    d = small_data
    p_rows, missing = synth.make_completeness(d.prep.row_pix, d.wl.nside, d.grid)
    o_cat = copy.copy(d.o_cat)
    o_cat.p_compl = {int(px): p_rows[i] for i, px in enumerate(d.prep.row_pix)}
    o_cat.missing = missing
    ctx, many = chimera.context_from_prepared(d.prep, d.inj)
    sets = {"many1d": many, "single1d": ctx.add_prepared_single1d(prep.single1d(d.prep, d.ev)),
            "3d": ctx.add_prepared_3d(prep.three_d(d.prep, d.ev))}
    lam = synth.make_lambdas(synth.WORKLOADS["precision_300ev"], batch=5, child=150)
    lam[0] = synth.LAMBDA_TRUTH
    plain = {k: ctx.lnl(v, lam, chimera.CHIMERA_FP64, with_lnI=True) for k, v in sets.items()}
    ctx.set_completeness(p_rows, missing)
    yield d, chimera, ctx, sets, o_cat, lam, plain, p_rows, missing
    ctx.close()


@pytest.mark.parametrize("kernel,shape", [("many1d", "gaussian"), ("single1d", "gaussian"),
                                          ("many1d", "epanechnikov"), ("3d", "gaussian")])
def test_matches_oracle(setup, kernel, shape):
    import oracle
    d, chimera, ctx, sets, o_cat, lam, plain, p_rows, missing = setup
    ev = sets[kernel]
    if shape != "gaussian":
        ctx.set_event_kde(ev, chimera.CHIMERA_KDE_EPANECHNIKOV, 0)
    try:
        lnl, lnI = ctx.lnl(ev, lam, chimera.CHIMERA_FP64, with_lnI=True)
        l32 = ctx.lnl(ev, lam, chimera.CHIMERA_FP32)
    finally:
        ctx.set_event_kde(ev)
    fin = np.isfinite(lnl)
    assert fin.sum() >= 2 and np.array_equal(np.isfinite(l32), fin)
    assert np.max(np.abs(l32[fin] - lnl[fin])) <= 1e-3
    # the completion changes the values
    assert np.max(np.abs(lnI[fin] - plain[kernel][1][fin])) > 1e-3
    for b in range(lam.shape[0]):
        ref = oracle.likelihood.lnl(d.o_events, o_cat, d.o_inj, lam[b], T=8.6, kernel=kernel,
                                    shape=shape)
        assert close(lnl[b], ref["lnl"], REL64), (b, lnl[b], ref["lnl"])
        for i in range(lnI.shape[1]):
            assert close(lnI[b, i], ref["lnI"][i], REL64), (b, i, lnI[b, i], ref["lnI"][i])


def test_selection_matches_oracle(setup):
    import oracle
    d, chimera, ctx, sets, o_cat, lam, plain, p_rows, missing = setup
    lx, ne = ctx.selection(lam, chimera.CHIMERA_FP64)
    for b in range(lam.shape[0]):
        xi, neff, _ = oracle.likelihood.selection(d.o_inj, o_cat, lam[b])
        if np.isfinite(lx[b]):
            assert abs(lx[b] - math.log(xi)) <= 1e-12 * max(1.0, abs(math.log(xi)))
            assert abs(ne[b] - neff) <= 1e-9 * neff


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
def test_gradient_matches_oracle(setup, kernel):
    """The adjoint with the incomplete catalogue against the oracle's gradient
    (1e-8) on the 10-event data."""
    from oracle import gradient as G
    d, chimera, ctx, sets, o_cat, lam, plain, p_rows, missing = setup
    lnl, grad = ctx.lnl_grad(sets[kernel], lam[:3], chimera.CHIMERA_FP64)
    for b in range(3):
        ref = G.lnl_grad(d.o_events, o_cat, d.o_inj, lam[b], T=8.6, kernel=kernel)
        if not np.isfinite(ref["lnl"]):
            assert not np.isfinite(lnl[b])
            continue
        assert close(lnl[b], ref["lnl"], REL64), (b, lnl[b], ref["lnl"])
        err = np.abs(grad[b] - ref["grad"]) / np.maximum(1.0, np.abs(ref["grad"]))
        assert np.all(err <= 1e-8), (b, err)


def test_cleared_gives_the_complete_catalogue_bitwise_and_refusals(setup):
    d, chimera, ctx, sets, o_cat, lam, plain, p_rows, missing = setup
    bad = p_rows.copy()
    bad[0, 3] = 1.5
    with pytest.raises(chimera.ChimeraError) as ex:
        ctx.set_completeness(bad, missing)
    assert ex.value.status == chimera.CHIMERA_EINVAL
    ctx.set_completeness(None)
    try:
        for k, ev in sets.items():
            lnl, lnI = ctx.lnl(ev, lam, chimera.CHIMERA_FP64, with_lnI=True)
            assert np.array_equal(lnl, plain[k][0], equal_nan=True), k
            assert np.array_equal(lnI, plain[k][1], equal_nan=True), k
        ctx.lnl_grad(sets["many1d"], lam[:2], chimera.CHIMERA_FP64)
    finally:
        ctx.set_completeness(p_rows, missing)


def test_empty_and_full_completeness_limits(setup):
    """P_compl = 0 everywhere (every row is the completion density alone) and
    P_compl = 1 (the catalogue rows times f_R) against the oracle (1e-10)."""
    import oracle
    d, chimera, ctx, sets, o_cat, lam, plain, p_rows, missing = setup
    area = synth.pixel_area(d.wl.nside)
    npix = 12 * d.wl.nside ** 2
    try:
        for val in (0.0, 1.0):
            pr = np.full_like(p_rows, val)
            ms = np.full(missing.shape, 4.0 * math.pi * (1.0 - val))
            ctx.set_completeness(pr, ms)
            lnl, lnI = ctx.lnl(sets["many1d"], lam[:2], chimera.CHIMERA_FP64, with_lnI=True)
            c = copy.copy(o_cat)
            c.p_compl = {k: np.full(d.grid.size, val) for k in o_cat.p_compl}
            c.missing = ms
            for b in range(2):
                ref = oracle.likelihood.lnl(d.o_events, c, d.o_inj, lam[b], T=8.6)
                assert close(lnl[b], ref["lnl"], REL64), (val, b, lnl[b], ref["lnl"])
                for i in range(lnI.shape[1]):
                    assert close(lnI[b, i], ref["lnI"][i], REL64), (val, b, i)
    finally:
        ctx.set_completeness(p_rows, missing)
    assert area * npix == pytest.approx(4.0 * math.pi, rel=1e-12)
