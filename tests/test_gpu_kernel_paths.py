"""The event kernel's less common paths against the oracle.  Direct sums: on a
20 000-point grid the Gaussian table of a wide event (windows over the whole
grid, about 40 000 entries) does not fit the workgroup's LDS, so its units
take direct sums in both precisions, while the narrow event of the same call
takes the Horner sweep.  Groups whose windows share no grid point: a
handmade event whose group spread cap is wide and bandwidth small.  The
largest events the library accepts: 2560 pixel rows (FP32 stages them two
grid points per slice; FP64 takes direct sums) and 2048 rows (FP64 stages
them one grid point per slice)."""
import numpy as np
import pytest

from tests.datasets import handcrafted_oracle
from tests.test_gpu_grad import hand_lams, wide_windows

pytestmark = pytest.mark.gpu

REL64 = 1e-10
ABS32 = 1e-3


def context(chimera, h, **kw):
    ctx = chimera.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"], **kw)
    ctx.set_catalog(h["rows"], h["nz_tot"])
    ctx.set_injections(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
    es = ctx.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"], h["dl"],
                        h["m1"], h["m2"])
    return ctx, es


def check(chimera, ctx, es, h, lam, T):
    import oracle
    events, cat, inj = handcrafted_oracle(h)
    l64, lnI64 = ctx.lnl(es, lam, chimera.CHIMERA_FP64, with_lnI=True)
    l32 = ctx.lnl(es, lam, chimera.CHIMERA_FP32)
    for b in range(lam.shape[0]):
        ref = oracle.likelihood.lnl(events, cat, inj, lam[b], T=T)
        print(b, l64[b], l32[b], ref["lnl"])
        assert np.isfinite(ref["lnl"])
        assert abs(l64[b] - ref["lnl"]) <= REL64 * abs(ref["lnl"])
        assert np.allclose(lnI64[b], ref["lnI"], rtol=REL64, atol=0.0)
        assert abs(l32[b] - ref["lnl"]) <= ABS32


def test_direct_sum_fallback_on_a_fine_grid():
    from paper_2504_02034_amd import chimera
    h = wide_windows()
    n_z = 20000
    grid = np.linspace(h["z_lo"], h["z_hi"], n_z)
    rows = np.stack([np.exp(-0.5 * ((grid - mu) / 0.05) ** 2) + 0.05 for mu in (0.4, 0.8, 1.1)])
    h.update(n_z=n_z, grid=grid, rows=rows, nz_tot=rows.mean(axis=0))
    ctx, es = context(chimera, h)
    check(chimera, ctx, es, h, hand_lams()[:2], T=8.6)
    ctx.close()


def masked_case():
    """One event: 40 zero-weight samples (masses above the support) in two far
    distance clusters widen the group spread cap (0.6 of the event's distance
    spread); 8 weighted samples 250 Mpc apart in one pixel; 200 weighted
    samples concentrated at 3700 Mpc keep the bandwidth small.  Groups of the
    middle pixel span more than 2 T h, so their windows share no grid point."""
    rng = np.random.default_rng(21)
    n_z, z_lo, z_hi = 1000, 0.0, 1.6
    grid = np.linspace(z_lo, z_hi, n_z)
    rows = np.stack([np.exp(-0.5 * ((grid - mu) / 0.05) ** 2) + 0.05 for mu in (0.4, 0.6, 0.8)])
    counts = np.array([40, 8, 200])
    dl = np.concatenate([np.linspace(1000.0, 1500.0, 20), np.linspace(11000.0, 11500.0, 20),
                         3000.0 + 250.0 * np.arange(8),
                         3700.0 * (1 + 0.003 * rng.standard_normal(200))])
    m1 = np.concatenate([np.full(40, 400.0), rng.uniform(30, 50, 208)])
    m2 = np.concatenate([np.full(40, 300.0), m1[40:] * rng.uniform(0.5, 0.9, 208)])
    ninj = 3000
    im1 = rng.uniform(8, 150, ninj)
    return dict(n_z=n_z, z_lo=z_lo, z_hi=z_hi, grid=grid, rows=rows, nz_tot=rows.mean(axis=0),
                ev_pix_off=np.array([0, 3]), pix_samp_off=np.concatenate([[0], np.cumsum(counts)]),
                pix_row=np.array([0, 1, 2]), c_ir=np.array([0.5, 0.3, 0.8]), dl=dl, m1=m1, m2=m2,
                idl=rng.uniform(100, 9000, ninj), im1=im1, im2=im1 * rng.uniform(0.2, 1.0, ninj),
                lnp=np.full(ninj, -12.0), ninj=ninj * 4)


def test_groups_without_a_common_window():
    """FP64 takes the fully masked sweep for such groups (or the direct sums
    where the chain range bound is exceeded), FP32 the direct sums."""
    import oracle
    from paper_2504_02034_amd import chimera
    h = masked_case()
    lam = hand_lams()[:3]
    # the weighted samples of the middle pixel are further apart than 2 T h
    events, _, _ = handcrafted_oracle(h)
    d = np.concatenate([p.dl for p in events[0].pixels])
    m1 = np.concatenate([p.m1d for p in events[0].pixels])
    m2 = np.concatenate([p.m2d for p in events[0].pixels])
    for b in range(lam.shape[0]):
        z, w = oracle.likelihood.redshift_and_weight(d, m1, m2, lam[b])
        hb = oracle.likelihood.bandwidth(z, w, h["grid"][1] - h["grid"][0])
        mid = z[40:48][w[40:48] > 0]
        assert mid.size >= 2 and mid.max() - mid.min() > 2 * 8.6 * hb
    ctx, es = context(chimera, h)
    check(chimera, ctx, es, h, lam, T=8.6)
    ctx.close()


def many_rows_case():
    """Event 0 over CHIMERA_MAX_EVENT_PIXELS = 2560 pixel rows, event 1 over
    2048, one to three samples per row, distances around 3000 Mpc."""
    rng = np.random.default_rng(31)
    n_z, z_lo, z_hi = 200, 0.0, 1.6
    grid = np.linspace(z_lo, z_hi, n_z)
    n_rows = 2560
    mu = rng.uniform(0.2, 1.2, n_rows)
    rows = np.exp(-0.5 * ((grid[None, :] - mu[:, None]) / 0.15) ** 2) + 0.02
    pix_row = np.concatenate([np.arange(n_rows), rng.permutation(n_rows)[:2048]])
    counts = rng.integers(1, 4, pix_row.size)
    S = int(counts.sum())
    dl = 3000.0 * (1 + 0.12 * rng.standard_normal(S))
    m1 = rng.uniform(20, 60, S)
    ninj = 3000
    im1 = rng.uniform(8, 150, ninj)
    return dict(n_z=n_z, z_lo=z_lo, z_hi=z_hi, grid=grid, rows=rows, nz_tot=rows.mean(axis=0),
                ev_pix_off=np.array([0, n_rows, pix_row.size]),
                pix_samp_off=np.concatenate([[0], np.cumsum(counts)]), pix_row=pix_row,
                c_ir=rng.uniform(0.2, 1.0, pix_row.size), dl=dl, m1=m1,
                m2=m1 * rng.uniform(0.5, 0.95, S), idl=rng.uniform(100, 9000, ninj), im1=im1,
                im2=im1 * rng.uniform(0.2, 1.0, ninj), lnp=np.full(ninj, -12.0), ninj=ninj * 4)


def test_events_with_the_most_pixel_rows():
    from paper_2504_02034_amd import chimera
    h = many_rows_case()
    assert h["ev_pix_off"][1] == chimera.CHIMERA_MAX_EVENT_PIXELS
    ctx, es = context(chimera, h)
    check(chimera, ctx, es, h, hand_lams()[:2], T=8.6)
    ctx.close()
