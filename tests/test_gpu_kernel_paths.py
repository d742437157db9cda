"""The event kernel's direct-sum fallback against the oracle: on a
20 000-point grid the Gaussian table of a wide event (windows over the whole
grid, about 40 000 entries) does not fit the workgroup's LDS, so its units
take direct sums in both precisions, while the narrow event of the same call
takes the Horner sweep."""
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
