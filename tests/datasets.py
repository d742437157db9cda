"""Seeded datasets shared by the tests (raw inputs from the generator, then
each side's own preprocessing)."""
import functools

import numpy as np

from paper_2504_02034_amd import prep, synth


class Data:
    pass


def build(wl, n_events=None, n_samples=None, oracle_side=True, rows_all=False):
    import oracle
    cf = synth.make_catalog(wl)
    ev = synth.make_events(wl, cf, n_events=n_events, n_samples=n_samples)
    inj = synth.make_injections(wl)
    d = Data()
    d.wl, d.cat, d.ev, d.inj = wl, cf[0], ev, inj
    d.grid = synth.z_grid(wl)
    d.area = synth.pixel_area(wl.nside)
    d.lam = synth.make_lambdas(wl)
    d.prep = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred)
    if oracle_side:
        d.o_events = oracle.prep.events(ev.offsets, ev.dl, ev.m1d, ev.m2d, ev.theta, ev.phi,
                                        ev.pix, lambda p: synth.pix2ang_ring(wl.nside, p),
                                        d.area, cred=wl.cred)
        rows_pix = sorted({px.pix for e in d.o_events for px in e.pixels})
        d.o_cat = oracle.prep.catalog(cf[0].z_obs, cf[0].pix, cf[0].sigma_z0, d.grid,
                                      np.asarray(rows_pix), d.area)
        d.o_inj = oracle.likelihood.InjectionSet(inj.dl, inj.m1d, inj.m2d, inj.ln_pdraw,
                                                 inj.n_total)
    return d


@functools.lru_cache(maxsize=None)
def small():
    return build(synth.WORKLOADS["fp64_10ev"])


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


def handcrafted_oracle(h):
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


def oracle_from_prepared(p, nz, nz_tot, inj, events=None):
    """Oracle structures over prepared arrays and a catalogue given as rows (the
    preprocessing output is data shared by both sides)."""
    import oracle
    L = oracle.likelihood
    grid = p.z_lo + (p.z_hi - p.z_lo) / (p.n_z - 1) * np.arange(p.n_z)
    out = []
    for e in (range(p.n_events) if events is None else events):
        ev = L.Event()
        for q in range(p.ev_pix_off[e], p.ev_pix_off[e + 1]):
            sl = slice(p.pix_samp_off[q], p.pix_samp_off[q + 1])
            ev.pixels.append(L.Pixel(pix=int(p.pix_row[q]), c=float(p.c_ir[q]), dl=p.dl[sl],
                                     m1d=p.m1d[sl], m2d=p.m2d[sl]))
        out.append(ev)
    rows = sorted({px.pix for ev in out for px in ev.pixels})
    cat = L.Catalog(grid=grid, rows={r: nz[r] for r in rows}, n_tot=nz_tot)
    o_inj = L.InjectionSet(inj.dl, inj.m1d, inj.m2d, inj.ln_pdraw, inj.n_total)
    return out, cat, o_inj
