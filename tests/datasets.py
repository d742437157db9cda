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
