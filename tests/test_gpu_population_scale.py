"""The paper-complete population and catalogue at the bench size: the
300-event workload with an incomplete catalogue and the smoothed lower mass
edge together, through the C-ABI.  FP64 ln I_i against the oracle at 1e-10 on
sampled events (event 104 is one of the lightest, far down the edge) at two
points; FP32 within 1e-3 of FP64, with the same finite mask, on 32 points of
the bench batch with delta_m from Table 1's prior U(0.01, 10)."""
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


def test_full_size_sampled_events():
    import oracle
    from paper_2504_02034_amd import chimera
    from tests.datasets import build
    d = build(synth.WORKLOADS["precision_300ev"])
    p_rows, missing = synth.make_completeness(d.prep.row_pix, d.wl.nside, d.grid)
    rng = np.random.default_rng(np.random.SeedSequence([250402034, 31]))
    lam = np.column_stack([d.lam[:32], rng.uniform(0.01, 10.0, 32)])
    lam[0, :14] = synth.LAMBDA_TRUTH
    lam[0, 14] = 4.8
    lam[1, 14] = 9.5
    ctx, es = chimera.context_from_prepared(d.prep, d.inj)
    try:
        ctx.set_completeness(p_rows, missing)
        ctx.set_mass_smoothing(True)
        lnl, lnI = ctx.lnl(es, lam, chimera.CHIMERA_FP64, with_lnI=True)
        l32 = ctx.lnl(es, lam, chimera.CHIMERA_FP32)
    finally:
        ctx.close()
    fin = np.isfinite(lnl)
    assert fin.sum() >= 8 and np.array_equal(np.isfinite(l32), fin)
    dmax = float(np.max(np.abs(l32[fin] - lnl[fin])))
    print("finite", int(fin.sum()), "max |dlnL| fp32 vs fp64", dmax)
    assert dmax <= 1e-3
    o_cat = copy.copy(d.o_cat)
    o_cat.p_compl = {int(px): p_rows[i] for i, px in enumerate(d.prep.row_pix)}
    o_cat.missing = missing
    evs = [0, 104, 299]
    for b in (0, 1):
        ref = oracle.likelihood.lnl(d.o_events, o_cat, d.o_inj, lam[b], T=8.6, event_subset=evs)
        for i in evs:
            assert np.isfinite(ref["lnI"][i])
            assert close(lnI[b, i], ref["lnI"][i], REL64), (b, i, lnI[b, i], ref["lnI"][i])
