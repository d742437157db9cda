"""The continuous-batching server on the device: requests from concurrent
clients over two resident event sets and both precisions, fused and
overlapped on several streams under an HBM budget that binds, each result
equal (bitwise) to the same request evaluated alone."""
import threading

import numpy as np
import pytest

from paper_2504_02034_amd import synth
from tests.datasets import handcrafted

pytestmark = pytest.mark.gpu


def test_served_results_equal_the_request_alone():
    from paper_2504_02034_amd import chimera
    from paper_2504_02034_amd.server import HipExecutor, Server
    h = handcrafted()
    ctx = chimera.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"])
    ctx.set_catalog(h["rows"], h["nz_tot"])
    ctx.set_injections(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
    full = ctx.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"], h["dl"],
                          h["m1"], h["m2"])
    k = h["pix_samp_off"][h["ev_pix_off"][2]]
    part = ctx.add_events(h["ev_pix_off"][:3], h["pix_samp_off"][:h["ev_pix_off"][2] + 1],
                          h["pix_row"][:h["ev_pix_off"][2]], h["c_ir"][:h["ev_pix_off"][2]],
                          h["dl"][:k], h["m1"][:k], h["m2"][:k])
    ex = HipExecutor(ctx)
    budget = 3 * ex.scratch_bytes(full, 48, chimera.CHIMERA_FP64)
    srv = Server(ex, n_workers=4, max_fused=48, hbm_budget=budget)
    rng0 = np.random.default_rng(11)
    base = synth.LAMBDA_TRUTH
    reqs, lock = [], threading.Lock()

    def client(seed):
        rng = np.random.default_rng(seed)
        for _ in range(12):
            B = int(rng.integers(1, 25))
            lam = np.tile(base, (B, 1))
            lam[:, 0] = rng.uniform(40, 120, B)
            lam[:, 1] = rng.uniform(0.1, 0.6, B)
            lam[:, 2] = rng.uniform(0.5, 2.5, B)
            lam[:, 3] = rng.uniform(0, 6, B)
            if rng.random() < 0.1:
                lam[0, 1] = 2.0            # an invalid point inside a request
            ev = full if rng.random() < 0.6 else part
            prec = int(rng.integers(2))
            t = srv.submit(ev, lam, prec)
            with lock:
                reqs.append((t, ev, lam, prec))

    th = [threading.Thread(target=client, args=(s,)) for s in range(5)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t, ev, lam, prec in reqs:
        got = srv.wait(t, timeout=120)
        alone = ctx.lnl(ev, lam, prec)
        assert np.array_equal(got, alone, equal_nan=True), (t.id, got, alone)
    st = srv.stats()
    srv.close()
    print(st)
    assert st["completed"] == len(reqs) == 60
    assert st["peak_bytes"] <= budget
    assert st["launches"] <= len(reqs)
    ctx.close()
