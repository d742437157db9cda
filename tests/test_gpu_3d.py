"""The 3D kernel (one Gaussian KDE of the samples in redshift and sky,
Sect. 2.2) through the C-ABI (chimera_add_events_3d) against the oracle:
per-event ln I_i on the 10-event workload and on sampled events of the
300-event workload, the FP32 form against FP64, the allocation-free entry
point, and the calls that refuse a 3D set."""
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


def prior_batch(n, seed):
    lam = synth.make_lambdas(synth.WORKLOADS["precision_300ev"], batch=n, child=100 + seed)
    lam[0] = synth.LAMBDA_TRUTH
    return lam


def context_3d(d):
    from paper_2504_02034_amd import chimera, prep
    ctx = chimera.Context(n_z=d.prep.n_z, z_lo=d.prep.z_lo, z_hi=d.prep.z_hi)
    ctx.set_catalog(d.prep.nz, d.prep.nz_tot)
    ctx.set_injections(d.inj.dl, d.inj.m1d, d.inj.m2d, d.inj.ln_pdraw, d.inj.n_total)
    t = prep.three_d(d.prep, d.ev)
    return chimera, ctx, ctx.add_prepared_3d(t), t


@pytest.fixture(scope="module")
def small3(small_data):
    chimera, ctx, es, t = context_3d(small_data)
    yield small_data, chimera, ctx, es, t
    ctx.close()


def test_fp64_matches_oracle(small3):
    import oracle
    d, chimera, ctx, es, t = small3
    lam = prior_batch(4, 12)
    lnl, lnI = ctx.lnl(es, lam, chimera.CHIMERA_FP64, with_lnI=True)
    l32 = ctx.lnl(es, lam, chimera.CHIMERA_FP32)
    fin = np.isfinite(lnl)
    assert fin.sum() >= 2 and np.array_equal(np.isfinite(l32), fin)
    d32 = np.max(np.abs(l32[fin] - lnl[fin]))
    print("max |dlnL| fp32-fp64", d32)
    assert d32 <= 1e-3
    for b in range(lam.shape[0]):
        ref = oracle.likelihood.lnl(d.o_events, d.o_cat, d.o_inj, lam[b], T=8.6, kernel="3d")
        print(b, lnl[b], ref["lnl"])
        assert close(lnl[b], ref["lnl"], REL64), (b, lnl[b], ref["lnl"])
        for i in range(lnI.shape[1]):
            assert close(lnI[b, i], ref["lnI"][i], REL64), (b, i, lnI[b, i], ref["lnI"][i])


def test_static_entry_point_on_a_3d_set(small3):
    import torch
    d, chimera, ctx, es, t = small3
    lam = torch.from_numpy(prior_batch(5, 13)).cuda()
    for prec in (chimera.CHIMERA_FP32, chimera.CHIMERA_FP64):
        want = torch.empty(5, dtype=torch.float64, device="cuda")
        chimera.chimera_lnl_batch(ctx.handle, es.handle, lam, prec, lnl=want)
        got = chimera.chimera_lnl_batch_static(ctx.handle, es.handle, lam, prec)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want.cpu().numpy(), equal_nan=True)


def test_refusals_and_argument_checks(small3):
    d, chimera, ctx, es, t = small3
    with pytest.raises(chimera.ChimeraError) as ex:
        ctx.lnl_grad(es, prior_batch(2, 14), chimera.CHIMERA_FP64)
    assert ex.value.status == chimera.CHIMERA_EINVAL
    with pytest.raises(chimera.ChimeraError) as ex:
        ctx.set_event_kde(es, chimera.CHIMERA_KDE_EPANECHNIKOV, 0)
    assert ex.value.status == chimera.CHIMERA_EINVAL
    ctx.set_event_kde(es)                       # the defaults are accepted
    args = [t.ev_samp_off, t.dl, t.m1d, t.m2d, t.sky_u, t.sky_v, t.ev_pix_off, t.pix_row, t.pix_u,
            t.pix_v, t.pix_area]

    def bad(i, v, status):
        a = list(args)
        a[i] = v
        with pytest.raises(chimera.ChimeraError) as e:
            ctx.add_events_3d(*a)
        assert e.value.status == status

    area = t.pix_area.copy()
    area[2] = 0.0
    bad(10, area, chimera.CHIMERA_EINVAL)
    rows = t.pix_row.copy()
    rows[1] = d.prep.nz.shape[0]
    bad(7, rows, chimera.CHIMERA_ERANGE)
    su = t.sky_u.copy()
    su[5] = np.nan
    bad(4, su, chimera.CHIMERA_EINVAL)
    po = t.ev_pix_off.copy()
    po[1] = 0
    bad(6, po, chimera.CHIMERA_EINVAL)


def test_full_size_sampled_events():
    """The 300-event workload at 8 lambda points (each launch holds about
    1e8 (pixel, sample) points per point, so the batch runs in chunks)."""
    import oracle
    from tests.datasets import build
    d = build(synth.WORKLOADS["precision_300ev"])
    chimera, ctx, es, t = context_3d(d)
    try:
        lam = d.lam[:8]
        lnl, lnI = ctx.lnl(es, lam, chimera.CHIMERA_FP64, with_lnI=True)
        l32 = ctx.lnl(es, lam, chimera.CHIMERA_FP32)
    finally:
        ctx.close()
    fin = np.isfinite(lnl)
    assert np.array_equal(np.isfinite(l32), fin)
    if fin.any():
        dmax = float(np.max(np.abs(l32[fin] - lnl[fin])))
        print("finite", int(fin.sum()), "max |dlnL| fp32 vs fp64", dmax)
        assert dmax <= 1e-3
    evs = [0, 151, 299]
    for b in (0, 5):
        ref = oracle.likelihood.lnl(d.o_events, d.o_cat, d.o_inj, lam[b], T=8.6,
                                    event_subset=evs, kernel="3d")
        for i in evs:
            assert close(lnI[b, i], ref["lnI"][i], REL64), (b, i, lnI[b, i], ref["lnI"][i])
