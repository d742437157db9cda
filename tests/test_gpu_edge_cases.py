"""Degenerate and edge inputs through the C-ABI, against the oracle on the
same handcrafted arrays: single-sample events and pixels, events whose
samples all fall outside the mass support, the alpha = 1 and beta = -1
special forms, lambda_g in {0, 1}, Xi0 = 1, no detected injections."""
import math

import numpy as np
import pytest

from paper_2504_02034_amd import synth

pytestmark = pytest.mark.gpu


def handcrafted():
    """Four events; event 0: one pixel with one sample; event 1: two pixels,
    one of them with a single sample; event 2: many samples in two pixels;
    event 3: one sample of non-zero weight whose distance group holds seven
    zero-weight samples far away in redshift (bandwidth at its floor, so the
    zero-weight chains would grow without bound if they were run)."""
    rng = np.random.default_rng(5)
    n_z, z_lo, z_hi = 400, 0.0, 1.6
    grid = np.linspace(z_lo, z_hi, n_z)
    rows = np.stack([np.exp(-0.5 * ((grid - mu) / 0.02) ** 2) + 0.05
                     for mu in (0.3, 0.5, 0.55, 0.9, 1.2)])
    nz_tot = rows.mean(axis=0)
    ev_pix_off = np.array([0, 1, 3, 5, 7])
    counts = np.array([1, 7, 1, 40, 33, 20, 8])
    pix_samp_off = np.concatenate([[0], np.cumsum(counts)])
    pix_row = np.array([0, 1, 2, 3, 4, 3, 2])
    c_ir = np.array([1.0, 0.13, 0.9, 0.02, 0.025, 0.04, 0.3])
    n = int(pix_samp_off[-1])
    base = np.repeat([1500.0, 2900.0, 2900.0, 5800.0, 5800.0, 0.0, 0.0], counts)
    dl = base * (1 + 0.08 * rng.standard_normal(n))
    m1 = rng.uniform(20, 60, n)
    m2 = m1 * rng.uniform(0.4, 1.0, n)
    e3 = slice(pix_samp_off[5], pix_samp_off[7])
    dl[e3] = np.concatenate([np.linspace(1000.0, 9000.0, 20), np.linspace(3500.0, 4700.0, 8)])
    m1[e3] = 400.0
    m2[e3] = 300.0
    j = pix_samp_off[6]
    m1[j], m2[j] = 40.0, 30.0
    ninj = 3000
    idl = rng.uniform(100, 9000, ninj)
    im1 = rng.uniform(8, 150, ninj)
    im2 = im1 * rng.uniform(0.2, 1.0, ninj)
    lnp = np.full(ninj, -12.0)
    return dict(n_z=n_z, z_lo=z_lo, z_hi=z_hi, grid=grid, rows=rows, nz_tot=nz_tot,
                ev_pix_off=ev_pix_off, pix_samp_off=pix_samp_off, pix_row=pix_row, c_ir=c_ir,
                dl=dl, m1=m1, m2=m2, idl=idl, im1=im1, im2=im2, lnp=lnp, ninj=ninj * 4)


def oracle_structs(h):
    import oracle
    L = oracle.likelihood
    events = []
    for e in range(len(h["ev_pix_off"]) - 1):
        ev = L.Event()
        for p in range(h["ev_pix_off"][e], h["ev_pix_off"][e + 1]):
            sl = slice(h["pix_samp_off"][p], h["pix_samp_off"][p + 1])
            ev.pixels.append(L.Pixel(pix=int(h["pix_row"][p]), c=float(h["c_ir"][p]),
                                     dl=h["dl"][sl], m1d=h["m1"][sl], m2d=h["m2"][sl]))
        events.append(ev)
    cat = L.Catalog(grid=h["grid"], rows={i: h["rows"][i] for i in range(len(h["rows"]))},
                    n_tot=h["nz_tot"])
    inj = L.InjectionSet(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
    return events, cat, inj


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
