"""Continuous-batching server for ln L requests from many concurrent samplers.

submit(events, lam [B, width], prec) -> Ticket; wait(ticket) -> ln L [B];
submit(..., grad=True) -> a gradient request; wait -> (ln L [B], d ln L [B, 12])
(the adjoint, for gradient-based samplers); stats() -> evals/s, p50 / p99
latency and admission figures.  Gradient requests are fused only with
gradient requests, and admitted by the gradient call's scratch.

The event sets, the catalogue and the injections stay resident in the
library's context.  Worker threads, each with its own HIP stream and its own
preallocated pinned and device buffers, take work as they free up:

* continuous batching: a free worker takes the oldest pending request and,
  with it, every other pending request on the same event set and precision
  (in arrival order) up to `max_fused` lambda points, and evaluates them in
  one call; each point's result does not depend on the others in its batch
  (every per-lambda reduction has a fixed order), so a request gets the same
  numbers alone and in any mix;
* admission by HBM budget: the library keeps one scratch block per stream,
  grown to the largest call made on it, so the memory held is the sum of
  the workers' blocks.  A worker takes a group only while that sum, with its
  own block grown to the group's need (chimera_scratch_bytes), stays within
  `hbm_budget`; when it would not, the blocks of idle workers are released
  (chimera_release_scratch) first;
* passing: when the oldest request cannot get memory, a later request that
  can may run first, as long as the oldest has waited less than `max_pass_s`
  (0: never pass; the oldest then waits for memory);
* short requests first: with `small_bytes` > 0 a request whose scratch need
  is at most that is small; a free worker takes the oldest small request
  before any other (fused only with small ones), and the first `reserved`
  workers take small requests only, so a short request never waits behind
  more than the small work in flight, however long the large requests are
  (a large request that has waited `large_age_s` goes before small ones);
* work of different workers overlaps on the device (one stream each).

The executor is pluggable: HipExecutor runs the library; tests of the
scheduling logic use a CPU stand-in.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Ticket:
    id: int
    events: object
    lam: np.ndarray
    prec: int
    t_submit: float
    need: int = 0
    small: bool = False
    t_start: float = 0.0
    t_done: float = 0.0
    grad: bool = False
    result: object = None
    error: BaseException = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def B(self) -> int:
        return self.lam.shape[0]


class HipExecutor:
    """Runs fused requests through chimera_lnl_batch on a per-worker stream,
    with per-worker pinned host and device buffers for lambda and ln L (no
    allocation per request).  chunk_bytes > 0 cuts a batch into launch
    sequences of at most that much per-point scratch (about that much work),
    enqueued back to back on the worker's stream: the device then interleaves
    other streams' kernels between them, so a short request does not wait for
    a whole large batch's kernels.  Each point's result does not depend on the
    chunking."""

    class Worker:
        def __init__(self, torch, max_fused):
            self.stream = torch.cuda.Stream()
            # flat, so that [B, width] views are contiguous for either lambda width
            self.lam_h = torch.empty(max_fused * 15, dtype=torch.float64, pin_memory=True)
            self.out_h = torch.empty(max_fused, dtype=torch.float64, pin_memory=True)
            self.lam_d = torch.empty(max_fused * 15, dtype=torch.float64, device="cuda")
            self.out_d = torch.empty(max_fused, dtype=torch.float64, device="cuda")
            # gradient requests: d ln L per point (12 parameters)
            self.grad_h = torch.empty(max_fused, 12, dtype=torch.float64, pin_memory=True)
            self.grad_d = torch.empty(max_fused, 12, dtype=torch.float64, device="cuda")
            self.done = torch.cuda.Event()

    def __init__(self, ctx, max_fused: int = 512, chunk_bytes: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.max_fused = max_fused
        self.chunk_bytes = chunk_bytes

    @property
    def lam_width(self) -> int:
        """Entries per lambda row (14, or 15 with the smoothed mass edge)."""
        return self.ctx.lam_width

    def new_worker(self):
        return HipExecutor.Worker(self.torch, self.max_fused)

    def scratch_bytes(self, events, B, prec, grad: bool = False) -> int:
        from . import chimera
        if grad:
            return self.ctx.grad_scratch_bytes(events, B, prec, chimera.CHIMERA_DEVICE)
        return self.ctx.scratch_bytes(events, B, prec, chimera.CHIMERA_DEVICE)

    def release(self, worker):
        self.ctx.release_scratch(worker.stream)

    def run(self, worker, events, lam, prec, grad: bool = False):
        """ln L [B], or (ln L [B], gradient [B, 12]) for a gradient request."""
        from . import chimera
        torch = self.torch
        B, W = lam.shape
        lam_h = worker.lam_h[:B * W].view(B, W)
        lam_d = worker.lam_d[:B * W].view(B, W)
        lam_h.copy_(torch.from_numpy(lam))
        step = B
        if self.chunk_bytes > 0 and B > 1:
            one = self.scratch_bytes(events, 1, prec, grad)
            per = max(self.scratch_bytes(events, 2, prec, grad) - one, 1)
            step = max(1, min(B, int(self.chunk_bytes // per)))
        with torch.cuda.stream(worker.stream):
            lam_d.copy_(lam_h, non_blocking=True)
            for i in range(0, B, step):
                if grad:
                    chimera.chimera_lnl_grad(self.ctx.handle, events.handle, lam_d[i:i + step],
                                             prec, lnl=worker.out_d[i:i + step],
                                             grad=worker.grad_d[i:i + step], stream=worker.stream)
                else:
                    self.ctx.lnl(events, lam_d[i:i + step], prec, lnl=worker.out_d[i:i + step],
                                 stream=worker.stream)
            worker.out_h[:B].copy_(worker.out_d[:B], non_blocking=True)
            if grad:
                worker.grad_h[:B].copy_(worker.grad_d[:B], non_blocking=True)
            worker.done.record(worker.stream)
        worker.done.synchronize()
        if grad:
            return worker.out_h[:B].numpy().copy(), worker.grad_h[:B].numpy().copy()
        return worker.out_h[:B].numpy().copy()


class Server:
    def __init__(self, executor, n_workers: int = 4, max_fused: int = 512,
                 hbm_budget: int = 0, max_pass_s: float = 0.0, small_bytes: int = 0,
                 reserved: int = 0, large_age_s: float = 1.0):
        if n_workers < 1 or max_fused < 1:
            raise ValueError("n_workers and max_fused must be >= 1")
        if reserved < 0 or reserved >= n_workers or (reserved and small_bytes <= 0):
            raise ValueError("reserved workers need small_bytes > 0 and one general worker")
        self.ex = executor
        self.max_fused = max_fused
        self.budget = int(hbm_budget)          # 0: no limit
        self.max_pass_s = float(max_pass_s)
        self.small_bytes = int(small_bytes)    # 0: no short-first ordering
        self.reserved = int(reserved)
        self.large_age_s = float(large_age_s)
        self._mu = threading.Lock()
        self._cv = threading.Condition(self._mu)
        self._pending: collections.deque = collections.deque()
        self._next_id = 0
        self._stop = False
        self._worker_objs = [self.ex.new_worker() for _ in range(n_workers)]
        self._arena = [0] * n_workers          # scratch block held by each worker's stream
        self._busy = [False] * n_workers
        # statistics
        self._lat = []
        self._evals = 0
        self._launches = 0
        self._fused_requests = 0
        self._passed = 0
        self._releases = 0
        self._peak_bytes = 0
        self._peak_inflight = 0
        self._inflight = 0
        self._t0 = None
        self._t_last = None
        self._workers = [threading.Thread(target=self._loop, args=(w,), daemon=True)
                         for w in range(n_workers)]
        for w in self._workers:
            w.start()

    # ------------------------------------------------------------------
    def _need(self, events, B, prec, grad) -> int:
        return (self.ex.scratch_bytes(events, B, prec, grad=True) if grad
                else self.ex.scratch_bytes(events, B, prec))

    def submit(self, events, lam, prec: int = 0, grad: bool = False) -> Ticket:
        lam = np.ascontiguousarray(np.atleast_2d(lam), dtype=np.float64)
        width = getattr(self.ex, "lam_width", 14)
        if lam.ndim != 2 or lam.shape[1] != width or lam.shape[0] < 1:
            raise ValueError(f"lam must be [B, {width}] with B >= 1")
        if lam.shape[0] > self.max_fused:
            raise ValueError(f"B = {lam.shape[0]} exceeds max_fused = {self.max_fused}")
        grad = bool(grad)
        if grad and width != 14:
            raise ValueError("the adjoint takes the unsmoothed mass model (14-wide lambda rows)")
        need = self._need(events, lam.shape[0], prec, grad)
        if self.budget and need > self.budget:
            raise MemoryError(f"request needs {need} bytes, over the budget of {self.budget}")
        with self._cv:
            if self._stop:
                raise RuntimeError("server is closed")
            t = Ticket(self._next_id, events, lam, prec, time.perf_counter(), need=need,
                       small=0 < need <= self.small_bytes if self.small_bytes else False,
                       grad=grad)
            self._next_id += 1
            if self._t0 is None:
                self._t0 = t.t_submit
            self._pending.append(t)
            self._cv.notify_all()
        return t

    def wait(self, ticket: Ticket, timeout=None):
        if not ticket.done.wait(timeout):
            raise TimeoutError(f"request {ticket.id} not done")
        if ticket.error is not None:
            raise ticket.error
        return ticket.result

    def stats(self) -> dict:
        with self._mu:
            lat = np.array(self._lat) * 1e3
            span = (self._t_last - self._t0) if self._t_last is not None else 0.0
            return {
                "completed": len(self._lat),
                "evals": self._evals,
                "evals_per_s": self._evals / span if span > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else float("nan"),
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else float("nan"),
                "launches": self._launches,
                "requests_per_launch": self._fused_requests / max(self._launches, 1),
                "passed": self._passed,
                "releases": self._releases,
                "peak_bytes": self._peak_bytes,
                "peak_inflight": self._peak_inflight,
                "budget": self.budget,
            }

    def reset_stats(self):
        """Forget the statistics so far (e.g. after a warm-up request)."""
        with self._mu:
            self._lat, self._evals, self._launches, self._fused_requests = [], 0, 0, 0
            self._passed, self._releases = 0, 0
            self._peak_bytes, self._peak_inflight = sum(self._arena), self._inflight
            self._t0, self._t_last = None, None

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for w in self._workers:
            w.join()

    # ------------------------------------------------------------------
    def _fits(self, w, need) -> bool:
        """Under the lock: can worker w run a call of `need` scratch bytes,
        releasing idle workers' blocks if that makes room?  A reserved
        worker's block counts as at least small_bytes and is never released,
        so the short requests always have their memory."""
        if not self.budget:
            return True
        held = sum(self._held(v) for v in range(len(self._arena)) if v != w)
        held += max(self._held(w), need)
        if held <= self.budget:
            return True
        for v in range(self.reserved, len(self._arena)):
            if held <= self.budget:
                break
            if v != w and not self._busy[v] and self._arena[v] > 0:
                self.ex.release(self._worker_objs[v])
                held -= self._arena[v]
                self._arena[v] = 0
                self._releases += 1
        return held <= self.budget

    def _held(self, v) -> int:
        return max(self._arena[v], self.small_bytes) if v < self.reserved else self._arena[v]

    def _group(self, head):
        group, B = [head], head.B
        for t in self._pending:
            if t is not head and t.events is head.events and t.prec == head.prec \
                    and t.small == head.small and t.grad == head.grad \
                    and B + t.B <= self.max_fused:
                group.append(t)
                B += t.B
        return group, B

    def _take(self, w):
        """Under the lock: the fused group for free worker w, or None."""
        if not self._pending:
            return None
        now = time.perf_counter()
        oldest = self._pending[0]
        may_pass = self.max_pass_s > 0 and now - oldest.t_submit < self.max_pass_s
        if self.small_bytes:
            # small requests first, except large ones that have waited past
            # large_age_s (so a stream of short requests cannot starve them)
            aged = [t for t in self._pending
                    if not t.small and now - t.t_submit > self.large_age_s]
            order = [] if w < self.reserved else list(aged)
            order += [t for t in self._pending if t.small]
            if w >= self.reserved:
                order += [t for t in self._pending if not t.small and t not in aged]
            if not order:
                return None
            if order[0] is not oldest:          # a small request goes first by rule, not by memory
                oldest = order[0]
                may_pass = self.max_pass_s > 0 and now - oldest.t_submit < self.max_pass_s
        else:
            order = list(self._pending)
        seen = set()
        for head in order:
            key = (id(head.events), head.prec, head.small, head.grad)
            if key in seen:
                continue
            seen.add(key)
            group, B = self._group(head)
            need = self._need(head.events, B, head.prec, head.grad)
            while len(group) > 1 and not self._fits(w, need):
                B -= group.pop().B
                need = self._need(head.events, B, head.prec, head.grad)
            if self._fits(w, need):
                for t in group:
                    self._pending.remove(t)
                if head is not oldest:
                    self._passed += 1
                return group, B, need
            if not may_pass:
                return None
        return None

    def _loop(self, w):
        worker = self._worker_objs[w]
        while True:
            with self._cv:
                while True:
                    got = self._take(w)
                    if got is not None or (self._stop and not self._pending):
                        break
                    self._cv.wait(timeout=self.max_pass_s if self.max_pass_s > 0 else None)
                if got is None:
                    return
                group, B, need = got
                self._arena[w] = max(self._arena[w], need)
                self._busy[w] = True
                self._inflight += 1
                self._peak_bytes = max(self._peak_bytes, sum(self._arena))
                self._peak_inflight = max(self._peak_inflight, self._inflight)
            t_start = time.perf_counter()
            lam = np.concatenate([t.lam for t in group]) if len(group) > 1 else group[0].lam
            err, out = None, None
            try:
                if group[0].grad:
                    out = self.ex.run(worker, group[0].events, lam, group[0].prec, grad=True)
                else:
                    out = self.ex.run(worker, group[0].events, lam, group[0].prec)
            except BaseException as e:  # noqa: BLE001 - handed to the waiting caller
                err = e
            t_done = time.perf_counter()
            with self._cv:
                self._busy[w] = False
                self._inflight -= 1
                self._launches += 1
                self._fused_requests += len(group)
                off = 0
                for t in group:
                    t.t_start, t.t_done = t_start, t_done
                    if err is None:
                        if t.grad:
                            t.result = (out[0][off:off + t.B].copy(), out[1][off:off + t.B].copy())
                        else:
                            t.result = out[off:off + t.B].copy()
                        self._lat.append(t_done - t.t_submit)
                        self._evals += t.B
                    else:
                        t.error = err
                    off += t.B
                    t.done.set()
                self._t_last = t_done
                self._cv.notify_all()
