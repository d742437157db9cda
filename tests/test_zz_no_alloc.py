"""The allocation-free entry point (chimera_lnl_batch_static) through the
C-ABI against chimera_lnl_batch in device mode: the same ln L and ln I_i,
bitwise, on two calls in a row, the second with a smaller batch, in both
precisions; on the 10-event workload (one launch sequence) and on the
300-event workload (the static scratch holds a few points, so the batch runs
as several launch sequences)."""
import numpy as np
import pytest

from paper_2504_02034_amd import synth

pytestmark = pytest.mark.gpu


def contexts():
    from paper_2504_02034_amd import chimera, prep
    for name, n_events in (("fp64_10ev", None), ("precision_300ev", None)):
        wl = synth.WORKLOADS[name]
        cf = synth.make_catalog(wl)
        ev = synth.make_events(wl, cf, n_events=n_events)
        inj = synth.make_injections(wl)
        p = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred)
        ctx, es = chimera.context_from_prepared(p, inj, device=0)
        lam = synth.make_lambdas(wl.scaled(lam_kind="prior"), batch=64)
        yield name, ctx, es, p.n_events, lam


def test_static_entry_point_equals_the_allocating_one():
    import torch
    from paper_2504_02034_amd import chimera
    for name, ctx, es, E, lam_all in contexts():
        for prec in (chimera.CHIMERA_FP32, chimera.CHIMERA_FP64):
            for B in (37, 11):                      # two calls in a row, the second smaller
                lam = torch.from_numpy(np.ascontiguousarray(lam_all[:B])).cuda()
                want = torch.empty(B, dtype=torch.float64, device="cuda")
                want_I = torch.empty((B, E), dtype=torch.float64, device="cuda")
                chimera.chimera_lnl_batch(ctx.handle, es.handle, lam, prec, lnl=want, lnI=want_I)
                got_I = torch.full((B, E), 7.0, dtype=torch.float64, device="cuda")
                got = chimera.chimera_lnl_batch_static(ctx.handle, es.handle, lam, prec,
                                                       lnI=got_I)
                got2 = chimera.chimera_lnl_batch_static(ctx.handle, es.handle, lam, prec)
                torch.cuda.synchronize()
                w, g, g2 = want.cpu().numpy(), got.cpu().numpy(), got2.cpu().numpy()
                print(name, prec, B, "finite", np.isfinite(w).sum(), w[:3], g[:3])
                assert np.isfinite(w).any()
                assert np.array_equal(g, w, equal_nan=True), (name, prec, B)
                assert np.array_equal(g2, w, equal_nan=True), (name, prec, B)
                assert np.array_equal(got_I.cpu().numpy(), want_I.cpu().numpy(), equal_nan=True)
        ctx.close()
