"""Degenerate and edge inputs through the C-ABI, against the oracle on the
same handcrafted arrays: single-sample events and pixels, events whose
samples all fall outside the mass support, the alpha = 1 and beta = -1
special forms, lambda_g in {0, 1}, Xi0 = 1, no detected injections."""
import math

import numpy as np
import pytest

from paper_2504_02034_amd import synth

from tests.datasets import handcrafted, handcrafted_oracle as oracle_structs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hand():
    from paper_2504_02034_amd import chimera
    h = handcrafted()
    ctx = chimera.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"])
    ctx.set_catalog(h["rows"], h["nz_tot"])
    ctx.set_injections(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
    es = ctx.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"], h["dl"],
                        h["m1"], h["m2"])
    yield h, chimera, ctx, es
    ctx.close()


def lam_cases():
    t = synth.LAMBDA_TRUTH
    out = {}
    out["truth"] = t.copy()
    a = t.copy(); a[4] = 1.0; out["alpha=1"] = a
    bb = t.copy(); bb[5] = -1.0; out["beta=-1"] = bb
    l0 = t.copy(); l0[10] = 0.0; out["lambda_g=0"] = l0
    l1 = t.copy(); l1[10] = 1.0; out["lambda_g=1"] = l1
    gr = t.copy(); gr[2] = 1.0; gr[3] = 0.0; out["Xi0=1,n=0"] = gr
    mg = t.copy(); mg[2] = 2.5; mg[3] = 8.0; out["Xi0=2.5,n=8"] = mg
    ex = t.copy(); ex[6] = 70.0; ex[7] = 200.0; ex[8] = 100.0; out["support above samples"] = ex
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_handcrafted_cases(hand, prec):
    import oracle
    h, chimera, ctx, es = hand
    events, cat, inj = oracle_structs(h)
    cases = lam_cases()
    lam = np.stack(list(cases.values()))
    lnl, lnI = ctx.lnl(es, lam, prec, with_lnI=True)
    for b, name in enumerate(cases):
        ref = oracle.likelihood.lnl(events, cat, inj, lam[b], T=8.6)
        print(name, lnl[b], ref["lnl"], lnI[b], ref["lnI"])
        tol = 1e-10 if prec == 0 else 1e-4
        for i in range(len(h["ev_pix_off"]) - 1):
            r = ref["lnI"][i]
            if math.isinf(r):
                assert lnI[b, i] == r, (name, i)
            else:
                assert abs(lnI[b, i] - r) <= tol * max(1.0, abs(r)), (name, i, lnI[b, i], r)
        r = ref["lnl"]
        if math.isinf(r) or math.isnan(r):
            assert lnl[b] == r or (math.isnan(r) and math.isnan(lnl[b])), name
        else:
            assert abs(lnl[b] - r) <= tol * max(1.0, abs(r)), (name, lnl[b], r)


def test_no_detected_injections(hand):
    h, chimera, ctx, es = hand
    from paper_2504_02034_amd import chimera as ch
    c2 = ch.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"])
    c2.set_catalog(h["rows"], h["nz_tot"])
    c2.set_injections(np.empty(0), np.empty(0), np.empty(0), np.empty(0), 1000)
    e2 = c2.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"], h["dl"],
                       h["m1"], h["m2"])
    lam = synth.LAMBDA_TRUTH[None, :]
    assert c2.lnl(e2, lam)[0] == -np.inf
    lx, ne = c2.selection(lam)
    assert lx[0] == -np.inf and ne[0] == 0.0
    c2.close()
