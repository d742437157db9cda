"""The continuous-batching server on the device: requests from concurrent
clients over two resident event sets and both precisions, fused and
overlapped on several streams under an HBM budget that binds, first come
first served or short requests first (then with batches cut into launch
sequences of a few points), each result equal (bitwise) to the same request
evaluated alone, and the scratch the
library holds (and the device memory in use) within the budget.  Also: host
calls from two threads on one stream, each equal to the same call alone."""
import threading

import numpy as np
import pytest

from paper_2504_02034_amd import synth
from tests.datasets import handcrafted

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("short_first", [False, True], ids=["fifo", "short_first"])
def test_served_results_equal_the_request_alone(short_first):
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
    import torch
    ex = HipExecutor(ctx, max_fused=48)
    if short_first:      # launch sequences of about 5 points: the results must not change
        ex.chunk_bytes = 5 * (ex.scratch_bytes(full, 2, chimera.CHIMERA_FP64)
                              - ex.scratch_bytes(full, 1, chimera.CHIMERA_FP64))
    budget = 3 * ex.scratch_bytes(full, 48, chimera.CHIMERA_FP64)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    prio = {}
    if short_first:      # requests up to 8 points on the smaller set go first, one worker kept
        prio = dict(small_bytes=ex.scratch_bytes(part, 8, chimera.CHIMERA_FP64), reserved=1)
    srv = Server(ex, n_workers=4, max_fused=48, hbm_budget=budget, max_pass_s=0.01, **prio)
    held_max = [0]
    stop = threading.Event()

    def watch():
        # device memory in use beyond what the process held before the server
        while not stop.is_set():
            free, _ = torch.cuda.mem_get_info()
            held_max[0] = max(held_max[0], free0 - free)
            stop.wait(0.002)

    watcher = threading.Thread(target=watch, daemon=True)
    watcher.start()
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
    served = [srv.wait(t, timeout=120) for t, _, _, _ in reqs]
    st = srv.stats()
    srv.close()
    stop.set()
    watcher.join()
    held = ctx.scratch_held()
    for got, (t, ev, lam, prec) in zip(served, reqs):
        alone = ctx.lnl(ev, lam, prec)
        assert np.array_equal(got, alone, equal_nan=True), (t.id, got, alone)
    print(st, "held", held, "device peak", held_max[0], "budget", budget)
    assert st["completed"] == len(reqs) == 60
    assert st["peak_bytes"] <= budget
    assert held <= budget
    # the workers' pinned and device buffers (4 x 48 x 15 doubles) and the
    # allocators' rounding aside, device memory in use stays within the budget
    assert held_max[0] <= budget + (64 << 20)
    assert st["launches"] <= len(reqs)
    ctx.close()


def test_host_calls_from_two_threads_on_one_stream():
    """Host-memory calls run on the null stream; two threads calling at once
    with different lambda each get what the call alone gives."""
    from paper_2504_02034_amd import chimera
    h = handcrafted()
    ctx = chimera.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"])
    ctx.set_catalog(h["rows"], h["nz_tot"])
    ctx.set_injections(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
    es = ctx.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"], h["dl"],
                        h["m1"], h["m2"])
    rng = np.random.default_rng(3)
    lams = []
    for k in range(2):
        B = 40 + 23 * k                    # different sizes: the shared block regrows
        lam = np.tile(synth.LAMBDA_TRUTH, (B, 1))
        lam[:, 0] = rng.uniform(40, 120, B)
        lam[:, 2] = rng.uniform(0.5, 2.5, B)
        lams.append(lam)
    alone = [[ctx.lnl(es, lam, prec) for prec in (0, 1)] for lam in lams]
    out = [[None, None], [None, None]]
    errs = []

    def worker(k):
        try:
            for r in range(20):
                prec = r % 2
                got = ctx.lnl(es, lams[k], prec)
                if not np.array_equal(got, alone[k][prec], equal_nan=True):
                    out[k][prec] = got
                    return
        except BaseException as e:  # noqa: BLE001
            errs.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    ctx.close()
    assert not errs, errs
    assert all(o is None for row in out for o in row), out


def test_served_results_with_the_population_options():
    """With an incomplete catalogue and the smoothed mass edge the server takes
    lambda rows of 15 (delta_m last), refuses rows of 14, and each served
    result equals the request alone bitwise."""
    from paper_2504_02034_amd import chimera
    from paper_2504_02034_amd.server import HipExecutor, Server
    h = handcrafted()
    ctx = chimera.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"])
    ctx.set_catalog(h["rows"], h["nz_tot"])
    ctx.set_injections(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
    es = ctx.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"], h["dl"],
                        h["m1"], h["m2"])
    grid = np.linspace(h["z_lo"], h["z_hi"], h["n_z"])
    p_rows = np.stack([1.0 / (1.0 + np.exp((grid - (0.5 + 0.15 * r)) / 0.1))
                       for r in range(h["rows"].shape[0])])
    ctx.set_completeness(p_rows, 4.0 * np.pi * (0.2 + 0.6 / (1.0 + np.exp(-(grid - 0.8) / 0.2))))
    ctx.set_mass_smoothing(True)
    srv = Server(HipExecutor(ctx, max_fused=32), n_workers=3, max_fused=32)
    try:
        with pytest.raises(ValueError):
            srv.submit(es, np.tile(synth.LAMBDA_TRUTH, (2, 1)), 0)
        reqs, lock = [], threading.Lock()

        def client(seed):
            rng = np.random.default_rng(seed)
            for _ in range(8):
                B = int(rng.integers(1, 12))
                lam = np.tile(np.append(synth.LAMBDA_TRUTH, 4.8), (B, 1))
                lam[:, 0] = rng.uniform(40, 120, B)
                lam[:, 14] = rng.uniform(0.01, 10.0, B)
                prec = int(rng.integers(2))
                t = srv.submit(es, lam, prec)
                with lock:
                    reqs.append((t, lam, prec))

        th = [threading.Thread(target=client, args=(s,)) for s in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        served = [srv.wait(t, timeout=120) for t, _, _ in reqs]
    finally:
        srv.close()
    for got, (t, lam, prec) in zip(served, reqs):
        alone = ctx.lnl(es, lam, prec)
        assert np.array_equal(got, alone, equal_nan=True)
    assert np.isfinite(np.concatenate(served)).any()
    ctx.close()


@pytest.mark.parametrize("chunked", [False, True], ids=["whole", "chunked"])
def test_served_gradients_equal_the_request_alone(chunked):
    """Gradient requests (submit(..., grad=True)) from concurrent clients,
    mixed with ln L requests on the same event set: every served ln L and
    gradient bitwise equal to the same chimera_lnl_grad call alone, in both
    precisions, with the gradient calls' scratch (chimera_grad_scratch_bytes)
    inside the HBM budget, also with fused batches cut into launch sequences
    of one point each."""
    from paper_2504_02034_amd import chimera
    from paper_2504_02034_amd.server import HipExecutor, Server
    h = handcrafted()
    ctx = chimera.Context(n_z=h["n_z"], z_lo=h["z_lo"], z_hi=h["z_hi"])
    try:
        ctx.set_catalog(h["rows"], h["nz_tot"])
        ctx.set_injections(h["idl"], h["im1"], h["im2"], h["lnp"], h["ninj"])
        es = ctx.add_events(h["ev_pix_off"], h["pix_samp_off"], h["pix_row"], h["c_ir"],
                            h["dl"], h["m1"], h["m2"])
        P64, P32 = chimera.CHIMERA_FP64, chimera.CHIMERA_FP32
        ex = HipExecutor(ctx, max_fused=32)
        # (the pool rounds blocks up, so on this small set the sizes coincide)
        g1 = ex.scratch_bytes(es, 1, P64, grad=True)
        assert g1 > 0 and ex.scratch_bytes(es, 32, P64, grad=True) >= g1
        if chunked:
            ex.chunk_bytes = 1            # every point its own launch sequence
        srv = Server(ex, n_workers=3, max_fused=32,
                     hbm_budget=3 * ex.scratch_bytes(es, 32, P64, grad=True))
        rng = np.random.default_rng(11)
        base = synth.make_lambdas(synth.WORKLOADS["precision_300ev"], batch=60, child=77)
        base[:, 8:11] = synth.LAMBDA_TRUTH[8:11]
        reqs, lock = [], threading.Lock()

        def client(c):
            for r in range(4):
                B = int(rng.integers(1, 6))
                lam = base[rng.integers(0, base.shape[0], B)]
                prec = P64 if (c + r) % 2 == 0 else P32
                grad = (c + r) % 3 != 0
                t = srv.submit(es, lam, prec, grad=grad)
                with lock:
                    reqs.append((t, lam, prec, grad))

        threads = [threading.Thread(target=client, args=(c,)) for c in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        got = [(srv.wait(t, timeout=120), lam, prec, grad) for t, lam, prec, grad in reqs]
        st = srv.stats()
        srv.close()
        n_grad = 0
        for res, lam, prec, grad in got:
            if grad:
                n_grad += 1
                lnl, g = ctx.lnl_grad(es, lam, prec)
                assert np.array_equal(res[0], lnl, equal_nan=True)
                assert np.array_equal(res[1], g, equal_nan=True)
            else:
                assert np.array_equal(res, ctx.lnl(es, lam, prec), equal_nan=True)
        assert n_grad >= 4 and st["completed"] == len(got)
        assert st["peak_bytes"] <= st["budget"]
    finally:
        ctx.close()
