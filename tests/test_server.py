"""Scheduling logic of the continuous-batching server with a CPU stand-in
for the device executor: results routed to the right requests whatever the
fusion, the memory held (every worker's scratch block) never above the HBM
budget, idle blocks released to make room, fusion of queued requests on the
same event set, first-come order under memory pressure unless passing is
allowed (then bounded by the oldest request's age), errors isolated to their
requests, drain on close."""
import threading
import time

import numpy as np
import pytest

from paper_2504_02034_amd.server import Server


class Events:
    def __init__(self, tag):
        self.tag = tag


class MockExec:
    """CPU stand-in: each worker's 'stream' keeps a scratch block grown to its
    largest call, as the library does, until released."""

    def __init__(self, per_point_s=2e-4, fail_tag=None):
        self.per_point_s = per_point_s
        self.fail_tag = fail_tag
        self.mu = threading.Lock()
        self.arena = {}
        self.peak = 0
        self.releases = 0
        self.calls = []
        self.grad_calls = []

    def new_worker(self):
        return object()

    def scratch_bytes(self, events, B, prec, grad=False):
        return 1000 + (300 if grad else 100) * B

    def release(self, worker):
        with self.mu:
            self.arena[id(worker)] = 0
            self.releases += 1

    def run(self, worker, events, lam, prec, grad=False):
        need = self.scratch_bytes(events, lam.shape[0], prec, grad)
        with self.mu:
            self.arena[id(worker)] = max(self.arena.get(id(worker), 0), need)
            self.peak = max(self.peak, sum(self.arena.values()))
            self.calls.append((events.tag, lam.shape[0], prec, time.perf_counter()))
            if grad:
                self.grad_calls.append((events.tag, lam.shape[0], prec))
        time.sleep(lam.shape[0] * self.per_point_s)
        if self.fail_tag is not None and events.tag == self.fail_tag:
            raise ValueError("executor failure")
        if grad:
            return value(events, lam, prec), gradient(events, lam, prec)
        return value(events, lam, prec)


def value(events, lam, prec):
    return lam[:, 0] * 3.0 + lam[:, 5] + 1000.0 * events.tag + 0.5 * prec


def gradient(events, lam, prec):
    cols = list(range(6)) + list(range(8, 14))
    return lam[:, cols] * 2.0 + events.tag + 0.25 * prec


def lam_batch(rng, B):
    lam = np.tile(np.arange(14, dtype=float), (B, 1))
    lam[:, 0] = rng.normal(size=B)
    lam[:, 5] = rng.normal(size=B)
    return lam


def test_results_follow_their_requests_under_concurrency():
    ex = MockExec()
    srv = Server(ex, n_workers=3, max_fused=64)
    evs = [Events(0), Events(1), Events(2)]
    out = []
    lock = threading.Lock()

    def client(seed):
        rng = np.random.default_rng(seed)
        for _ in range(15):
            ev = evs[rng.integers(3)]
            prec = int(rng.integers(2))
            lam = lam_batch(rng, int(rng.integers(1, 20)))
            t = srv.submit(ev, lam, prec)
            with lock:
                out.append((t, ev, lam, prec))

    th = [threading.Thread(target=client, args=(s,)) for s in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t, ev, lam, prec in out:
        assert np.array_equal(srv.wait(t, timeout=30), value(ev, lam, prec))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(out)
    assert st["evals"] == sum(lam.shape[0] for _, _, lam, _ in out)
    assert st["launches"] <= len(out)
    assert st["p99_ms"] >= st["p50_ms"] > 0.0


def test_budget_is_never_exceeded_and_queued_requests_fuse():
    ex = MockExec(per_point_s=1e-3)
    budget = 2 * (1000 + 100 * 16)
    srv = Server(ex, n_workers=4, max_fused=16, hbm_budget=budget)
    ev = Events(0)
    rng = np.random.default_rng(1)
    ts = [(srv.submit(ev, lam, 0), lam) for lam in (lam_batch(rng, 4) for _ in range(24))]
    for t, lam in ts:
        assert np.array_equal(srv.wait(t, timeout=30), value(ev, lam, 0))
    st = srv.stats()
    srv.close()
    assert ex.peak <= budget and st["peak_bytes"] <= budget
    assert st["launches"] < len(ts)                     # queued requests were fused
    assert max(b for _, b, _, _ in ex.calls) <= 16


def test_fusion_keeps_event_sets_and_precisions_apart():
    ex = MockExec(per_point_s=2e-3)
    srv = Server(ex, n_workers=1, max_fused=512)
    rng = np.random.default_rng(2)
    blocker = srv.submit(Events(9), lam_batch(rng, 20), 0)     # keeps the worker busy
    a, b = Events(0), Events(1)
    reqs = [(srv.submit(e, lam, p), e, lam, p)
            for e, p in ((a, 0), (b, 0), (a, 1), (a, 0), (b, 0), (a, 1))
            for lam in [lam_batch(rng, 3)]]
    srv.wait(blocker, timeout=30)
    for t, e, lam, p in reqs:
        assert np.array_equal(srv.wait(t, timeout=30), value(e, lam, p))
    srv.close()
    groups = [(tag, B, prec) for tag, B, prec, _ in ex.calls[1:]]
    assert sorted(groups) == [(0, 6, 0), (0, 6, 1), (1, 6, 0)]


def test_oldest_request_is_not_passed_over_under_memory_pressure():
    ex = MockExec(per_point_s=5e-3)
    big = 1000 + 100 * 30
    srv = Server(ex, n_workers=3, max_fused=30, hbm_budget=big)
    rng = np.random.default_rng(3)
    first = srv.submit(Events(1), lam_batch(rng, 2), 0)        # runs at once
    time.sleep(0.002)
    large = srv.submit(Events(2), lam_batch(rng, 30), 0)       # must wait for memory
    later = [srv.submit(Events(1), lam_batch(rng, 2), 0) for _ in range(3)]
    for t in [first, large] + later:
        srv.wait(t, timeout=30)
    srv.close()
    assert all(t.t_start >= large.t_start for t in later)


def test_rejects_oversized_requests():
    srv = Server(MockExec(), n_workers=1, max_fused=8, hbm_budget=1500)
    rng = np.random.default_rng(4)
    with pytest.raises(ValueError):
        srv.submit(Events(0), lam_batch(rng, 9), 0)
    with pytest.raises(MemoryError):
        srv.submit(Events(0), lam_batch(rng, 8), 0)            # 1800 bytes > 1500
    with pytest.raises(ValueError):
        srv.submit(Events(0), np.zeros((2, 13)), 0)
    srv.close()


def test_executor_errors_stay_with_their_requests():
    ex = MockExec(fail_tag=7)
    srv = Server(ex, n_workers=2, max_fused=32)
    rng = np.random.default_rng(5)
    bad = srv.submit(Events(7), lam_batch(rng, 3), 0)
    good = [(srv.submit(Events(1), lam, 0), lam) for lam in (lam_batch(rng, 2) for _ in range(5))]
    with pytest.raises(ValueError):
        srv.wait(bad, timeout=30)
    for t, lam in good:
        assert np.array_equal(srv.wait(t, timeout=30), value(Events(1), lam, 0))
    srv.close()


def test_close_drains_pending_requests():
    srv = Server(MockExec(per_point_s=1e-3), n_workers=1, max_fused=4)
    rng = np.random.default_rng(6)
    ts = [srv.submit(Events(0), lam_batch(rng, 4), 0) for _ in range(5)]
    srv.close()
    assert all(t.done.is_set() and t.error is None for t in ts)
    with pytest.raises(RuntimeError):
        srv.submit(Events(0), lam_batch(rng, 1), 0)


def test_idle_blocks_are_released_to_make_room():
    """Admission counts the blocks every worker's stream holds: a call that
    would push the sum over the budget first releases idle workers' blocks
    (never a busy worker's), and is refused when that does not make room."""
    ex = MockExec()
    big = 1000 + 100 * 20
    srv = Server(ex, n_workers=3, max_fused=20, hbm_budget=big + 1200)
    w0, w1, w2 = srv._worker_objs
    with srv._cv:
        srv._arena[:] = [big, 0, 1100]
        srv._busy[:] = [False, False, True]
        assert srv._fits(1, big)                 # worker 0's idle block goes
        assert srv._arena == [0, 0, 1100] and ex.releases == 1
        srv._arena[:] = [0, big, 1100]
        srv._busy[:] = [False, True, True]
        assert not srv._fits(0, big)             # the busy blocks stay
        assert srv._arena == [0, big, 1100] and ex.releases == 1
        srv._arena[:] = [0, 0, 0]
        srv._busy[:] = [False, False, False]
    srv.close()
    # and end to end: large calls one after the other on whichever worker is
    # free never hold more than the budget
    ex = MockExec(per_point_s=1e-3)
    srv = Server(ex, n_workers=2, max_fused=20, hbm_budget=big + 1200)
    rng = np.random.default_rng(7)
    ts = [srv.submit(Events(0), lam_batch(rng, 20), 0) for _ in range(6)]
    for t in ts:
        srv.wait(t, timeout=30)
    st = srv.stats()
    srv.close()
    assert ex.peak <= big + 1200 and st["peak_bytes"] <= big + 1200


def test_passing_the_oldest_is_bounded_by_its_age():
    """With passing allowed, small requests run while the large oldest one
    waits for memory, and the large one still runs once its age bound is
    reached (no starvation under a steady stream of small requests)."""
    ex = MockExec(per_point_s=4e-3)
    big = 1000 + 100 * 30
    srv = Server(ex, n_workers=3, max_fused=30, hbm_budget=big, max_pass_s=0.05)
    rng = np.random.default_rng(8)
    first = srv.submit(Events(1), lam_batch(rng, 2), 0)        # holds memory for a while
    time.sleep(0.002)
    large = srv.submit(Events(2), lam_batch(rng, 30), 0)
    small = []
    t_end = time.perf_counter() + 0.4
    while time.perf_counter() < t_end:                          # a steady stream of small ones
        small.append(srv.submit(Events(1), lam_batch(rng, 2), 0))
        time.sleep(0.004)
    for t in [first, large] + small:
        srv.wait(t, timeout=30)
    st = srv.stats()
    srv.close()
    assert st["passed"] >= 1
    assert any(t.t_start < large.t_start for t in small)        # some passed the large one
    assert large.t_start - large.t_submit < 0.05 + 0.25          # bounded wait
    assert ex.peak <= big


def test_small_requests_overtake_large_ones():
    """With short-first ordering and one reserved worker, short requests
    submitted behind a queue of long ones finish long before the long ones,
    and the reserved worker never runs a long request."""
    ex = MockExec(per_point_s=2e-3)
    small_need = ex.scratch_bytes(None, 4, 0)
    srv = Server(ex, n_workers=2, max_fused=64, small_bytes=small_need, reserved=1,
                 large_age_s=60.0)
    big, little = Events(1), Events(2)
    rng = np.random.default_rng(3)
    longs = [srv.submit(big, lam_batch(rng, 60)) for _ in range(4)]
    time.sleep(0.01)
    shorts = [srv.submit(little, lam_batch(rng, 2)) for _ in range(6)]
    for t in longs + shorts:
        srv.wait(t, timeout=30)
    srv.close()
    assert max(t.t_done for t in shorts) < max(t.t_done for t in longs)
    lat_short = max(t.t_done - t.t_submit for t in shorts)
    assert lat_short < 60 * 2e-3 * 2            # well under two long requests
    assert all(t.small for t in shorts) and not any(t.small for t in longs)


def test_aged_large_requests_are_not_starved():
    """A long request that has waited past large_age_s goes before newer short
    ones: one worker, short requests arriving faster than it serves them (so
    short ones are always pending), and the long one still finishes soon."""
    ex = MockExec(per_point_s=1e-3)
    srv = Server(ex, n_workers=1, max_fused=32, small_bytes=ex.scratch_bytes(None, 2, 0),
                 large_age_s=0.02)
    big, little = Events(1), Events(2)
    rng = np.random.default_rng(4)
    stop = threading.Event()

    def flood():
        while not stop.is_set():
            srv.submit(little, lam_batch(rng, 1))
            time.sleep(0.0005)

    th = threading.Thread(target=flood)
    th.start()
    try:
        time.sleep(0.01)
        t_long = srv.submit(big, lam_batch(rng, 20))
        srv.wait(t_long, timeout=5.0)
    finally:
        stop.set()
        th.join()
        srv.close()
    assert t_long.t_done - t_long.t_submit < 0.5
    assert t_long.t_start - t_long.t_submit >= 0.02 * 0.5    # it did wait behind short ones


def test_priority_arguments_checked():
    ex = MockExec()
    with pytest.raises(ValueError):
        Server(ex, n_workers=2, reserved=1)           # reserved workers need small_bytes
    with pytest.raises(ValueError):
        Server(ex, n_workers=2, small_bytes=10, reserved=2)


def test_gradient_requests_fuse_only_with_gradient_requests():
    """Gradient requests (the adjoint) and ln L requests on the same event set
    and precision: each gets its own kind of result, they are fused only with
    their own kind, and their scratch is the gradient call's."""
    ex = MockExec(per_point_s=2e-3)
    srv = Server(ex, n_workers=1, max_fused=512)
    rng = np.random.default_rng(5)
    blocker = srv.submit(Events(9), lam_batch(rng, 20), 0)     # keeps the worker busy
    a = Events(0)
    reqs = [(srv.submit(a, lam, 0, grad=g), lam, g)
            for g in (True, False, True, False, True)
            for lam in [lam_batch(rng, 3)]]
    assert [t.need for t, _, _ in reqs] == [1900, 1300, 1900, 1300, 1900]
    srv.wait(blocker, timeout=30)
    for t, lam, g in reqs:
        got = srv.wait(t, timeout=30)
        if g:
            assert np.array_equal(got[0], value(a, lam, 0))
            assert np.array_equal(got[1], gradient(a, lam, 0))
        else:
            assert np.array_equal(got, value(a, lam, 0))
    srv.close()
    assert sorted(B for _, B, _, _ in ex.calls[1:]) == [6, 9]
    assert ex.grad_calls == [(0, 9, 0)]
    other = Server(MockExec(), n_workers=1)
    with pytest.raises(ValueError):
        other.submit(a, np.zeros((1, 15)), 0, grad=True)
    other.close()
