"""The kernel options of Sect. 2.3 through the C-ABI (chimera_set_event_kde):
the Epanechnikov kernel and binned data sets, on many-1D and single-1D sets,
against the oracle per event (FP64 1e-10), the FP32 form against FP64, the
allocation-free entry point, the return to the defaults, the degenerate bin
counts, the argument checks, and sampled events of the 300-event workload."""
import math

import numpy as np
import pytest

from paper_2504_02034_amd import synth

pytestmark = pytest.mark.gpu
REL64 = 1e-10
SHAPES = {"gaussian": 0, "epanechnikov": 1}
OPTIONS = [("epanechnikov", 0), ("gaussian", 16), ("epanechnikov", 16), ("gaussian", 5)]


def close(a, b, rel):
    if math.isnan(b):
        return math.isnan(a)
    if math.isinf(b):
        return a == b
    return abs(a - b) <= rel * max(1.0, abs(b))


def prior_batch(n, seed):
    lam = synth.make_lambdas(synth.WORKLOADS["precision_300ev"], batch=n, child=100 + seed)
    lam[0] = synth.LAMBDA_TRUTH
    return lam


@pytest.fixture(scope="module")
def sets(small_data):
    from paper_2504_02034_amd import chimera, prep
    d = small_data
    ctx, many = chimera.context_from_prepared(d.prep, d.inj)
    single = ctx.add_prepared_single1d(prep.single1d(d.prep, d.ev))
    yield d, chimera, ctx, {"many1d": many, "single1d": single}
    ctx.close()


@pytest.mark.parametrize("kernel", ["many1d", "single1d"])
@pytest.mark.parametrize("shape,n_bins", OPTIONS)
def test_fp64_matches_oracle(sets, kernel, shape, n_bins):
    import oracle
    d, chimera, ctx, es = sets
    ev = es[kernel]
    ctx.set_event_kde(ev, SHAPES[shape], n_bins)
    try:
        lam = prior_batch(6, 7)
        lnl, lnI = ctx.lnl(ev, lam, chimera.CHIMERA_FP64, with_lnI=True)
        l32 = ctx.lnl(ev, lam, chimera.CHIMERA_FP32)
    finally:
        ctx.set_event_kde(ev)
    fin = np.isfinite(lnl)
    assert fin.sum() >= 2 and np.array_equal(np.isfinite(l32), fin)
    d32 = np.max(np.abs(l32[fin] - lnl[fin]))
    print(kernel, shape, n_bins, "max |dlnL| fp32-fp64", d32)
    assert d32 <= 1e-3
    for b in range(lam.shape[0]):
        ref = oracle.likelihood.lnl(d.o_events, d.o_cat, d.o_inj, lam[b], T=8.6, kernel=kernel,
                                    shape=shape, n_bins=n_bins)
        assert close(lnl[b], ref["lnl"], REL64), (b, lnl[b], ref["lnl"])
        for i in range(lnI.shape[1]):
            assert close(lnI[b, i], ref["lnI"][i], REL64), (b, i, lnI[b, i], ref["lnI"][i])


def test_defaults_restored_bitwise(sets):
    d, chimera, ctx, es = sets
    ev = es["many1d"]
    lam = prior_batch(8, 8)
    before = ctx.lnl(ev, lam, chimera.CHIMERA_FP64)
    ctx.set_event_kde(ev, chimera.CHIMERA_KDE_EPANECHNIKOV, 12)
    other = ctx.lnl(ev, lam, chimera.CHIMERA_FP64)
    ctx.set_event_kde(ev)
    after = ctx.lnl(ev, lam, chimera.CHIMERA_FP64)
    assert np.array_equal(before, after, equal_nan=True)
    fin = np.isfinite(before) & np.isfinite(other)
    assert fin.any() and not np.array_equal(before[fin], other[fin])


def test_bin_counts_at_the_extremes(sets):
    """One bin: each pixel's weight at the centre of its range; more bins than
    samples: mostly empty bins.  Both against the oracle."""
    import oracle
    d, chimera, ctx, es = sets
    ev = es["many1d"]
    lam = prior_batch(3, 9)
    for nb in (1, chimera.CHIMERA_MAX_BINS):
        ctx.set_event_kde(ev, chimera.CHIMERA_KDE_GAUSSIAN, nb)
        try:
            lnl, lnI = ctx.lnl(ev, lam, chimera.CHIMERA_FP64, with_lnI=True)
        finally:
            ctx.set_event_kde(ev)
        for b in range(lam.shape[0]):
            ref = oracle.likelihood.lnl(d.o_events, d.o_cat, d.o_inj, lam[b], T=8.6, n_bins=nb)
            for i in range(lnI.shape[1]):
                assert close(lnI[b, i], ref["lnI"][i], REL64), (nb, b, i, lnI[b, i], ref["lnI"][i])


def test_static_entry_point_with_options(sets):
    import torch
    d, chimera, ctx, es = sets
    ev = es["single1d"]
    lam = torch.from_numpy(prior_batch(7, 10)).cuda()
    for shape, nb in OPTIONS:
        ctx.set_event_kde(ev, SHAPES[shape], nb)
        try:
            for prec in (chimera.CHIMERA_FP32, chimera.CHIMERA_FP64):
                want = torch.empty(7, dtype=torch.float64, device="cuda")
                chimera.chimera_lnl_batch(ctx.handle, ev.handle, lam, prec, lnl=want)
                got = chimera.chimera_lnl_batch_static(ctx.handle, ev.handle, lam, prec)
                torch.cuda.synchronize()
                assert np.array_equal(got.cpu().numpy(), want.cpu().numpy(), equal_nan=True)
        finally:
            ctx.set_event_kde(ev)


def test_argument_checks(sets):
    d, chimera, ctx, es = sets
    ev = es["many1d"]
    for shape, nb in ((2, 0), (-1, 0), (0, -1), (0, chimera.CHIMERA_MAX_BINS + 1)):
        with pytest.raises(chimera.ChimeraError) as ex:
            ctx.set_event_kde(ev, shape, nb)
        assert ex.value.status == chimera.CHIMERA_EINVAL
    ctx.lnl_grad(ev, prior_batch(2, 11), chimera.CHIMERA_FP64)


@pytest.fixture(scope="module")
def full():
    from tests.datasets import build
    from paper_2504_02034_amd import chimera, prep
    d = build(synth.WORKLOADS["precision_300ev"])
    ctx, many = chimera.context_from_prepared(d.prep, d.inj)
    single = ctx.add_prepared_single1d(prep.single1d(d.prep, d.ev))
    yield d, chimera, ctx, {"many1d": many, "single1d": single}
    ctx.close()


@pytest.mark.parametrize("kernel,shape,n_bins", [("many1d", "epanechnikov", 0),
                                                 ("many1d", "gaussian", 16),
                                                 ("single1d", "epanechnikov", 64)])
def test_full_size_sampled_events(full, kernel, shape, n_bins):
    import oracle
    d, chimera, ctx, es = full
    ev = es[kernel]
    ctx.set_event_kde(ev, SHAPES[shape], n_bins)
    try:
        lnl, lnI = ctx.lnl(ev, d.lam, chimera.CHIMERA_FP64, with_lnI=True)
        l32 = ctx.lnl(ev, d.lam, chimera.CHIMERA_FP32)
    finally:
        ctx.set_event_kde(ev)
    fin = np.isfinite(lnl)
    assert np.array_equal(np.isfinite(l32), fin)
    dmax = float(np.max(np.abs(l32[fin] - lnl[fin])))
    print(kernel, shape, n_bins, "finite", int(fin.sum()), "max |dlnL| fp32 vs fp64", dmax)
    assert dmax <= 1e-3
    rng = np.random.default_rng(13)
    evs = [0, 299] + list(rng.choice(np.arange(1, 299), 3, replace=False))
    for b in [0, 255] + list(rng.choice(np.arange(1, 255), 1, replace=False)):
        ref = oracle.likelihood.lnl(d.o_events, d.o_cat, d.o_inj, d.lam[b], T=8.6,
                                    event_subset=evs, kernel=kernel, shape=shape, n_bins=n_bins)
        for i in evs:
            assert close(lnI[b, i], ref["lnI"][i], REL64), (b, i, lnI[b, i], ref["lnI"][i])
