#!/usr/bin/env python3
"""Throughput of the batched ln L hot path on one MI355X.

One step = one chimera_lnl_batch call over a batch of lambda points: the
per-lambda distance tables, the grid factor, the injection sums (xi) and the
per-(event, lambda) kernel sums for every event, then ln L (the whole path).
Inputs are resident in HBM before the timed region; lambda stays on the
device and the call is asynchronous on torch's current stream.

Workload (default): 300 events x 5000 posterior samples, 1e6 spectroscopic
galaxies on HEALPix nside 64, 1000-point redshift grid, 1e6 injections, a
batch of 256 lambda drawn from the priors H0 in [20,140], Om in [0.1,0.5],
Xi0 in [0.3,3], n in [0,10].  Synthetic, seeded.

Prints one JSON line.  `value` is the FP32-bulk form's ln L evaluations per
second; the plain FP64 path is reported beside it with the FP32-FP64
|Delta lnL| of the same batch.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}     # MI355X published dense vector peaks
# FP32 without packed instructions (the build turns them off): one FMA per lane per cycle
PEAK_TFLOPS_UNPACKED = {"fp64": 78.6, "fp32": 78.6}
# algorithmic cost of one (sample, grid point) kernel evaluation: the Gaussian
# recurrence K_{g+1} = K_g r_g, r_{g+1} = r_g q and the multiply-add of K F
# into the sum, 4 flops (the kernels' Horner chains spend one FMA per pair)
FLOPS_PER_EVAL = 4.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(wl_name, batch):
    from paper_2504_02034_amd import prep, synth
    wl = synth.WORKLOADS[wl_name]
    t = time.time()
    cf = synth.make_catalog(wl)
    ev = synth.make_events(wl, cf)
    inj = synth.make_injections(wl)
    p = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred)
    lam = synth.make_lambdas(wl, batch=batch)
    log(f"inputs ready in {time.time() - t:.1f}s: {p.n_events} events, {p.dl.size} samples, "
        f"{p.nz.shape[0]} catalogue rows, {inj.dl.size} detected injections")
    return wl, cf, ev, inj, p, lam


def time_precision(ctx, es, lam_t, prec, steps, warmup):
    import torch
    from paper_2504_02034_amd import chimera
    out = torch.empty(lam_t.shape[0], dtype=torch.float64, device=lam_t.device)
    for _ in range(warmup):
        ctx.lnl(es, lam_t, prec, lnl=out)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        ctx.lnl(es, lam_t, prec, lnl=out)
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    # the dominant kernel, timed with HIP events on the same stream
    chimera.chimera_profile_enable(ctx.handle, True)
    for _ in range(steps):
        ctx.lnl(es, lam_t, prec, lnl=out)
    torch.cuda.synchronize()
    n, ms, evals = chimera.chimera_profile_read(ctx.handle)
    chimera.chimera_profile_enable(ctx.handle, False)
    return out.cpu().numpy(), wall, lat, n, ms, evals


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_event_kernels_precision_300ev.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_event_kernels_precision_300ev.json")


def current_summary(path, workload):
    """A committed counter summary (JSON), or None when it is absent, for
    another workload, or taken on sources that differ from the ones built now."""
    import hashlib
    if workload != "precision_300ev" or not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    h = hashlib.sha256()
    for src in t["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return t if h.hexdigest() == t["sources_sha256"] else None


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed traffic summary (or None)."""
    t = current_summary(TRAFFIC_FILE, workload)
    if t is None or kernel not in t["kernels"]:
        return None
    return t["kernels"][kernel]["traffic_bytes"]


def measured_counters(kernel, workload):
    """VALU lane instructions per evaluated pair and the VALU busy fraction of
    `kernel` from the committed instruction-counter summary (or None)."""
    t = current_summary(COUNTERS_FILE, workload)
    if t is None or kernel not in t["kernels"]:
        return None
    k = t["kernels"][kernel]
    return {"valu_lane_instr_per_pair": k["valu_lane_instr_per_pair"],
            "valu_busy": k["valu_busy"], "source": os.path.relpath(COUNTERS_FILE, ROOT)}


def pct(v, q):
    k = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def cpu_baseline(wl, cf, ev, inj, lams, n_events):
    """The oracle as it stands on this host: a few lambda points, a subset of
    events."""
    import numpy as np

    import oracle
    from paper_2504_02034_amd import synth
    grid = synth.z_grid(wl)
    area = synth.pixel_area(wl.nside)
    sub = synth.Events(offsets=ev.offsets[:n_events + 1], dl=ev.dl, m1d=ev.m1d, m2d=ev.m2d,
                       theta=ev.theta, phi=ev.phi, pix=ev.pix, nside=ev.nside)
    o_ev = oracle.prep.events(sub.offsets, sub.dl, sub.m1d, sub.m2d, sub.theta, sub.phi, sub.pix,
                              lambda q: synth.pix2ang_ring(wl.nside, q), area, cred=wl.cred)
    rows = sorted({px.pix for e in o_ev for px in e.pixels})
    o_cat = oracle.prep.catalog(cf[0].z_obs, cf[0].pix, cf[0].sigma_z0, grid, np.asarray(rows),
                                area)
    o_inj = oracle.likelihood.InjectionSet(inj.dl, inj.m1d, inj.m2d, inj.ln_pdraw, inj.n_total)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    t_sel = t_all = 0.0
    for lam in lams:
        t = time.perf_counter()
        oracle.likelihood.selection(o_inj, o_cat, lam)
        t_sel += time.perf_counter() - t
        t = time.perf_counter()
        oracle.likelihood.lnl(o_ev, o_cat, o_inj, lam, T=8.6, workers=cores)
        t_all += time.perf_counter() - t
    n = len(lams)
    t_ev = max(t_all - t_sel, 1e-9)
    per_lambda = (t_sel + t_ev * wl.n_events / n_events) / n
    return {"value": 1.0 / per_lambda, "unit": "lnL evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} lambda points of the batch with finite ln L, {n_events} of "
                      f"{wl.n_events} events (T=8.6 windows) plus the selection sum over all "
                      f"{inj.dl.size} detected injections; event time scaled by "
                      f"{wl.n_events}/{n_events}; measured {t_all:.1f}s"}


def grad_checks(ctx, es, lam_t, n_points=2):
    """At the full gradient workload: the FP32 adjoint's error against FP64 over
    every finite point, and the FP64 adjoint against central differences of
    the FP64 ln L (step 1e-5 relative, all 12 parameters) at a few points.
    ln L jumps where a source-frame mass crosses the mass model's hard edges
    inside the step: a (point, parameter) whose differences at steps h and h/2
    disagree by more than 10 % is counted as such and left out."""
    import numpy as np

    from paper_2504_02034_amd import chimera, synth
    lam = lam_t.cpu().numpy()
    l64, g64 = ctx.lnl_grad(es, lam, chimera.CHIMERA_FP64)
    _, g32 = ctx.lnl_grad(es, lam, chimera.CHIMERA_FP32)
    fin = np.flatnonzero(np.isfinite(l64))
    rel32 = np.abs(g32[fin] - g64[fin]) / np.maximum(1.0, np.abs(g64[fin]))
    def central(l, p, st):
        lp, lm = l.copy(), l.copy()
        lp[p] += st
        lm[p] -= st
        return (ctx.lnl(es, lp[None], chimera.CHIMERA_FP64)[0]
                - ctx.lnl(es, lm[None], chimera.CHIMERA_FP64)[0]) / (2 * st)

    worst, jumps, n = 0.0, 0, 0
    for b in fin[:: max(1, fin.size // n_points)][:n_points]:
        for kk, p in enumerate(synth.GRAD_COLUMNS):
            st = 1e-5 * abs(lam[b, p])
            fd, fd2 = central(lam[b], p, st), central(lam[b], p, 0.5 * st)
            n += 1
            if abs(fd - fd2) > 0.1 * max(1.0, abs(fd2)):
                jumps += 1
                continue
            worst = max(worst, abs(g64[b, kk] - fd) / max(1.0, abs(fd)))
    log(f"grad checks: FP32 vs FP64 max rel {rel32.max() if rel32.size else None}, "
        f"FP64 vs central differences max rel {worst:.2e} ({jumps} of {n} pairs with a jump)")
    return {"finite_points": int(fin.size),
            "fp32_vs_fp64_max_rel_err": float(rel32.max()) if rel32.size else None,
            "fp64_vs_central_difference": {"points": int(min(n_points, fin.size)),
                                           "step_rel": 1e-5, "pairs": n,
                                           "pairs_with_a_jump": jumps,
                                           "max_rel_err": float(worst)}}


def time_grad(ctx, es, lam_t, prec, steps):
    import torch
    ctx.lnl_grad(es, lam_t, prec)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        ctx.lnl_grad(es, lam_t, prec)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / steps


#: the other kernels of Sect. 2.3 timed on the same events: (KDE layout,
#: 1-D kernel shape, bins per KDE data set)
VARIANTS = [("single1d", "gaussian", 0), ("many1d", "epanechnikov", 0),
            ("single1d", "epanechnikov", 0), ("many1d", "gaussian", 16),
            ("single1d", "gaussian", 64), ("3d", "gaussian", 0)]
#: the 3D kernel does about (pixels per event) times the many-1D work per
#: point: it is timed on the first points of the batch
BATCH_3D = 16


def variants_bench(ctx, es, p, ev, lam_t, many, steps, warmup):
    """Each variant on the bench batch: ms per step in both precisions, the
    dominant kernel's time (HIP events), FP32 vs FP64 |Delta ln L| and the
    speedup over the many-1D Gaussian step of the same precision."""
    import numpy as np
    from paper_2504_02034_amd import chimera, prep
    shapes = {"gaussian": chimera.CHIMERA_KDE_GAUSSIAN,
              "epanechnikov": chimera.CHIMERA_KDE_EPANECHNIKOV}
    single = ctx.add_prepared_single1d(prep.single1d(p, ev))
    three = ctx.add_prepared_3d(prep.three_d(p, ev))
    sets = {"many1d": es, "single1d": single, "3d": three}
    out = []
    for kernel, shape, nb in VARIANTS:
        es_v = sets[kernel]
        ctx.set_event_kde(es_v, shapes[shape], nb)
        lam_v = lam_t[:BATCH_3D] if kernel == "3d" else lam_t
        B = lam_v.shape[0]
        r = {"kernel": kernel, "shape": shape, "n_bins": nb, "batch": B}
        vals = {}
        for name, prec in (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32)):
            o, wall, lat, n, ms, evals = time_precision(ctx, es_v, lam_v, prec, steps, warmup)
            avg_ms = ms / max(n, 1)
            dominant = ("k_event_epan" if shape == "epanechnikov" else "k_event_smooth") + name[2:]
            vals[name] = o
            # the many-1D step scaled to this batch (its cost is linear in the points)
            many_wall = many[name]["wall"] * B / lam_t.shape[0]
            r[name] = {"value": round(B * steps / wall, 2), "ms_per_step": round(wall / steps * 1e3, 4),
                       "kernel": dominant, "kernel_ms": round(avg_ms, 4),
                       "launches_per_step": round(n / steps, 2),
                       "speedup_over_many1d_gaussian": round(many_wall / wall, 4)}
            if shape == "gaussian":
                per_launch = evals / max(n, 1)
                achieved = per_launch * FLOPS_PER_EVAL / (avg_ms * 1e-3) / 1e12
                r[name].update(evals_per_launch=int(per_launch), achieved_tflops=round(achieved, 3),
                               frac=round(achieved / PEAK_TFLOPS[name], 4))
            else:
                r[name]["points_per_launch"] = int(evals / max(n, 1))
            log(f"{kernel} {shape} bins={nb} {name}: {wall / steps * 1e3:.2f} ms/step, "
                f"{dominant} {avg_ms:.2f} ms")
        fin = np.isfinite(vals["fp64"]) & np.isfinite(vals["fp32"])
        r["abs_dlnL_fp32_vs_fp64"] = {
            "max": float(np.max(np.abs(vals["fp32"][fin] - vals["fp64"][fin]))) if fin.any() else None,
            "same_finite_mask": bool(np.array_equal(np.isfinite(vals["fp32"]),
                                                    np.isfinite(vals["fp64"]))),
            "finite_points": int(fin.sum())}
        ctx.set_event_kde(es_v)
        out.append(r)
    single.release()
    three.release()
    return out


def population_bench(ctx, es, wl, p, lam_t, many, steps, warmup):
    """The many-1D Gaussian step with the paper-complete population and
    catalogue options on the bench batch: an incomplete catalogue (the
    generator's synthetic completeness), the smoothed lower mass edge with
    delta_m per point drawn from Table 1's prior U(0.01, 10), and both; ms per
    step and the main kernels' times in both precisions, FP32 vs FP64
    |Delta ln L|, and the cost over the plain step; with the incomplete
    catalogue also the gradient of the first 64 points against the plain
    gradient of the same points."""
    import numpy as np
    import torch

    from paper_2504_02034_amd import chimera, synth
    grid = np.linspace(wl.z_lo, wl.z_hi, wl.n_z)
    p_rows, missing = synth.make_completeness(p.row_pix, wl.nside, grid)
    rng = np.random.default_rng(np.random.SeedSequence([250402034, 77]))
    dm = torch.from_numpy(rng.uniform(0.01, 10.0, lam_t.shape[0])).to(lam_t.device)
    lam15 = torch.cat([lam_t, dm[:, None]], dim=1).contiguous()
    lam_g = lam_t[:64].contiguous()
    grad_plain = {n: time_grad(ctx, es, lam_g, p_, 3) for n, p_ in
                  (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32))}
    out = []
    for name in ("completeness", "mass_smoothing", "both"):
        if name != "mass_smoothing":
            ctx.set_completeness(p_rows, missing)
        if name != "completeness":
            ctx.set_mass_smoothing(True)
        lam_v = lam15 if name != "completeness" else lam_t
        r = {"option": name, "batch": int(lam_v.shape[0])}
        vals = {}
        try:
            for prec_name, prec in (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32)):
                o, wall, lat, n, ms, evals = time_precision(ctx, es, lam_v, prec, steps, warmup)
                vals[prec_name] = o
                r[prec_name] = {"value": round(lam_v.shape[0] * steps / wall, 2),
                                "ms_per_step": round(wall / steps * 1e3, 4),
                                "smooth_kernel_ms": round(ms / max(n, 1), 4),
                                "over_plain": round(wall / many[prec_name]["wall"], 4)}
                log(f"{name} {prec_name}: {wall / steps * 1e3:.2f} ms/step "
                    f"({wall / many[prec_name]['wall']:.3f} x plain)")
                if name == "completeness":
                    sec = time_grad(ctx, es, lam_g, prec, 3)
                    r[prec_name].update(grad_ms_64=round(sec * 1e3, 3),
                                        grad_over_plain=round(sec / grad_plain[prec_name], 4))
                    log(f"{name} {prec_name} gradient: {sec * 1e3:.2f} ms for 64 lambda "
                        f"({sec / grad_plain[prec_name]:.3f} x plain)")
        finally:
            ctx.set_completeness(None)
            ctx.set_mass_smoothing(False)
        fin = np.isfinite(vals["fp64"]) & np.isfinite(vals["fp32"])
        r["abs_dlnL_fp32_vs_fp64"] = {
            "max": float(np.max(np.abs(vals["fp32"][fin] - vals["fp64"][fin]))) if fin.any() else None,
            "same_finite_mask": bool(np.array_equal(np.isfinite(vals["fp32"]),
                                                    np.isfinite(vals["fp64"]))),
            "finite_points": int(fin.sum())}
        out.append(r)
    return out


def serve_bench(wl, cf, inj, n_requests=300, seed=5, max_pass_s=0.05, chunk_gb=4.0):
    """Serving: resident event sets of 50, 300, 1000 and 3000 distinct events
    x 4096 samples (nested subsets of one generated set of 3000) sharing the
    workload's catalogue and injections; a Poisson trace of requests, sizes
    log-uniform in 1..512, event set uniform.  First the FP32 server is
    saturated (every request queued at once) to measure its throughput; the
    open-loop trace then arrives at 0.7 of that rate.  The FP32 server
    (continuous batching, 4 streams, HBM budget, passing bounded by
    max_pass_s, short requests first with one worker kept for them) and plain
    FP64 launches, one request at a time, replay the same trace; each request
    is then timed alone, and its served latency over that time is its
    slowdown."""
    import numpy as np

    from paper_2504_02034_amd import chimera, prep, synth
    from paper_2504_02034_amd.server import HipExecutor, Server
    sizes = (50, 300, 1000, 3000)
    t = time.perf_counter()
    ev = synth.make_events(wl, cf, n_events=sizes[-1], n_samples=4096, child=6)
    p = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred)
    log(f"serving inputs ready in {time.perf_counter() - t:.1f}s: {p.n_events} events, "
        f"{p.dl.size} samples, {p.nz.shape[0]} catalogue rows")
    ctx, full = chimera.context_from_prepared(p, inj, device=0, n_tab=8192)
    sets = [ctx.add_prepared(prep.subset(p, list(range(n)))) for n in sizes[:-1]] + [full]
    rng = np.random.default_rng(seed)
    B = np.clip(np.floor(np.exp(rng.uniform(0.0, math.log(513.0), n_requests))).astype(int), 1, 512)
    which = rng.integers(0, len(sets), n_requests)
    base = synth.make_lambdas(synth.WORKLOADS["precision_300ev"])
    lams = [base[rng.integers(0, base.shape[0], b)] for b in B]
    gaps = rng.exponential(1.0, n_requests)
    ex = HipExecutor(ctx, max_fused=512, chunk_bytes=int(chunk_gb * (1 << 30)))
    biggest = max(ex.scratch_bytes(sets[w], int(b), chimera.CHIMERA_FP32) for b, w in zip(B, which))
    budget = int(2.5 * biggest)
    # short requests (up to the scratch of 128 points on the 300-event set) go
    # first, one worker serving only them
    small = ex.scratch_bytes(sets[1], 128, chimera.CHIMERA_FP32)
    srv = Server(ex, n_workers=4, max_fused=512, hbm_budget=budget, max_pass_s=max_pass_s,
                 small_bytes=small, reserved=1)
    srv.wait(srv.submit(sets[1], lams[0][:1], chimera.CHIMERA_FP32))      # warm up
    # saturated throughput: the whole trace queued at once
    srv.reset_stats()
    t0 = time.perf_counter()
    for t in [srv.submit(sets[which[i]], lams[i], chimera.CHIMERA_FP32) for i in range(n_requests)]:
        srv.wait(t)
    t_sat = time.perf_counter() - t0
    sat = srv.stats()
    rate = 0.7 * n_requests / t_sat                                   # requests per second
    arrivals = np.cumsum(gaps / rate)
    srv.reset_stats()
    tickets = []
    t0 = time.perf_counter()
    for i in range(n_requests):
        dt = arrivals[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(sets[which[i]], lams[i], chimera.CHIMERA_FP32))
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    held = ctx.scratch_held()
    # each request alone on an idle device (same executor path): the server's
    # latency over this service time is the request's slowdown
    solo = ex.new_worker()
    big = int(np.argmax([ex.scratch_bytes(sets[w], int(b), chimera.CHIMERA_FP32)
                         for b, w in zip(B, which)]))
    ex.run(solo, sets[which[big]], lams[big], chimera.CHIMERA_FP32)    # the stream's block, once
    alone = np.empty(n_requests)
    for i in range(n_requests):
        t1 = time.perf_counter()
        ex.run(solo, sets[which[i]], lams[i], chimera.CHIMERA_FP32)
        alone[i] = time.perf_counter() - t1
    lat32 = np.array([t.t_done - t.t_submit for t in tickets])
    is_small = np.array([t.small for t in tickets])
    wait32 = np.array([t.t_start - t.t_submit for t in tickets])
    run32 = np.array([t.t_done - t.t_start for t in tickets])
    slow = lat32 / alone
    per_set = {}
    for k, n in enumerate(sizes):
        m = which == k
        per_set[str(n)] = {"requests": int(m.sum()),
                           "p50_ms": round(float(np.percentile(lat32[m], 50)) * 1e3, 3),
                           "p99_ms": round(float(np.percentile(lat32[m], 99)) * 1e3, 3),
                           "alone_p99_ms": round(float(np.percentile(alone[m], 99)) * 1e3, 3)}
    # plain FP64 launches, one request at a time, same trace
    lat = []
    t0 = time.perf_counter()
    for i in range(n_requests):
        dt = arrivals[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ctx.lnl(sets[which[i]], lams[i], chimera.CHIMERA_FP64)
        lat.append(time.perf_counter() - t0 - arrivals[i])
    span64 = time.perf_counter() - t0
    lat = sorted(lat)
    # gradient requests (the adjoint through the server, for gradient-based
    # samplers): 64 requests of 1..8 points on the 300-event set at once,
    # against the same requests as one call each, one after another
    gsrv = Server(ex, n_workers=4, max_fused=512, hbm_budget=budget)
    g_b = rng.integers(1, 9, 64)
    g_lams = [base[rng.integers(0, base.shape[0], b)] for b in g_b]
    gsrv.wait(gsrv.submit(sets[1], g_lams[0][:1], chimera.CHIMERA_FP32, grad=True))  # warm up
    gsrv.reset_stats()
    t1 = time.perf_counter()
    for t in [gsrv.submit(sets[1], lg, chimera.CHIMERA_FP32, grad=True) for lg in g_lams]:
        gsrv.wait(t)
    g_span = time.perf_counter() - t1
    g_st = gsrv.stats()
    gsrv.close()
    t1 = time.perf_counter()
    for lg in g_lams:
        ctx.lnl_grad(sets[1], lg, chimera.CHIMERA_FP32)
    g_seq = time.perf_counter() - t1
    grad_serving = {"requests": 64, "points": int(g_b.sum()), "event_set": sizes[1],
                    "server_points_per_s": round(float(g_b.sum()) / g_span, 1),
                    "p50_ms": round(g_st["p50_ms"], 3), "p99_ms": round(g_st["p99_ms"], 3),
                    "requests_per_launch": round(g_st["requests_per_launch"], 3),
                    "one_call_each_points_per_s": round(float(g_b.sum()) / g_seq, 1)}
    log(f"serving gradients: {grad_serving['server_points_per_s']:.0f} points/s through the "
        f"server ({grad_serving['requests_per_launch']:.2f} requests per launch), "
        f"{grad_serving['one_call_each_points_per_s']:.0f} points/s one call each")
    ctx.close()
    log(f"serving: FP32 server p50 {st['p50_ms']:.1f} ms p99 {st['p99_ms']:.1f} ms, "
        f"{st['requests_per_launch']:.2f} requests per launch, slowdown over alone p50 "
        f"{np.percentile(slow, 50):.2f} p99 {np.percentile(slow, 99):.2f}")
    return {
        "gradient_requests": grad_serving,
        "requests": n_requests, "event_sets": list(sizes), "samples_per_event": 4096,
        "batch": "log-uniform 1..512",
        "saturated_fp32_evals_per_s": round(float(B.sum()) / t_sat, 1),
        "saturated_requests_per_launch": round(sat["requests_per_launch"], 3),
        "arrival_rate_req_s": round(rate, 2),
        "fp32_server": {"evals_per_s": round(st["evals_per_s"], 1),
                        "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                        "launches": st["launches"],
                        "requests_per_launch": round(st["requests_per_launch"], 3),
                        "passed": st["passed"], "scratch_releases": st["releases"],
                        "peak_inflight": st["peak_inflight"],
                        "peak_scratch_gb": round(st["peak_bytes"] / 2**30, 2),
                        "scratch_held_after_gb": round(held / 2**30, 2),
                        "hbm_budget_gb": round(budget / 2**30, 2),
                        "max_pass_ms": round(max_pass_s * 1e3, 1),
                        "launch_chunk_gb": chunk_gb,
                        "small_request_gb": round(small / 2**30, 3), "reserved_workers": 1,
                        "small_requests": int(is_small.sum()),
                        "small_wait_p99_ms": round(float(np.percentile(wait32[is_small], 99)) * 1e3, 3),
                        "small_run_p99_ms": round(float(np.percentile(run32[is_small], 99)) * 1e3, 3),
                        "small_latency_p99_ms": round(float(np.percentile(lat32[is_small], 99)) * 1e3, 3),
                        "slowdown_p50": round(float(np.percentile(slow, 50)), 3),
                        "slowdown_p99": round(float(np.percentile(slow, 99)), 3),
                        "alone_p50_ms": round(float(np.percentile(alone, 50)) * 1e3, 3),
                        "alone_p99_ms": round(float(np.percentile(alone, 99)) * 1e3, 3),
                        "per_event_set": per_set},
        "fp64_plain": {"evals_per_s": round(float(B.sum()) / span64, 1),
                       "p50_ms": round(pct(lat, 50) * 1e3, 3),
                       "p99_ms": round(pct(lat, 99) * 1e3, 3)},
    }


def photo_bench(xi0_truths=(1.0,), steps=3):
    """The photometric stress workload: 1000 events x 4096 samples, 1e7 photo-z
    galaxies (catalogue density built on the device), 2000-point grid to
    z = 2.4, 5e6 injections, B = 128; one event set and catalogue per Xi0 truth."""
    import numpy as np
    import torch

    from paper_2504_02034_amd import chimera, prep, synth
    out = []
    for k, xt in enumerate(xi0_truths):
        # Xi0 = 1 is the photo_1000ev workload itself; the other truths get seeds of their own
        seed = {1.0: 2, 0.6: 3, 1.8: 4}.get(xt, 5 + k)
        wl = synth.WORKLOADS["photo_1000ev"].scaled(xi0_truth=xt, seed_index=seed)
        cf = synth.make_catalog(wl)
        ev = synth.make_events(wl, cf)
        inj = synth.make_injections(wl)
        p = prep.prepare(cf[0], ev, wl.n_z, wl.z_lo, wl.z_hi, cred=wl.cred, with_catalog=False)
        gal = prep.galaxy_arrays(cf[0], wl.n_z, wl.z_lo, wl.z_hi)
        ctx = chimera.Context(n_z=wl.n_z, z_lo=wl.z_lo, z_hi=wl.z_hi)
        t = time.perf_counter()
        ctx.set_catalog_galaxies(*gal, p.row_pix)
        t_cat = time.perf_counter() - t
        ctx.set_injections(inj.dl, inj.m1d, inj.m2d, inj.ln_pdraw, inj.n_total)
        es = ctx.add_prepared(p)
        lam = torch.from_numpy(synth.make_lambdas(wl)).cuda()
        r = {"xi0_truth": xt, "samples": int(p.dl.size), "catalogue_rows": int(len(p.row_pix)),
             "catalogue_build_ms": round(t_cat * 1e3, 1)}
        vals = {}
        for name, prec in (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32)):
            ctx.lnl(es, lam, prec)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                v = ctx.lnl(es, lam, prec)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t) / steps
            vals[name] = v.cpu().numpy()
            r[name] = {"ms_per_step": round(sec * 1e3, 3), "evals_per_s": round(lam.shape[0] / sec, 1)}
        fin = np.isfinite(vals["fp64"]) & np.isfinite(vals["fp32"])
        r["abs_dlnL_fp32_vs_fp64"] = {
            "max": float(np.max(np.abs(vals["fp32"][fin] - vals["fp64"][fin]))) if fin.any() else None,
            "same_finite_mask": bool(np.array_equal(np.isfinite(vals["fp32"]), np.isfinite(vals["fp64"]))),
            "finite_points": int(fin.sum())}
        out.append(r)
        ctx.close()
        log(f"photo-z Xi0={xt}: fp64 {r['fp64']['ms_per_step']} ms, fp32 {r['fp32']['ms_per_step']} ms "
            f"per {lam.shape[0]} lambda; catalogue built in {r['catalogue_build_ms']} ms")
    return {"workload": "photo_1000ev", "events": 1000, "samples_per_event": 4096,
            "galaxies": 10_000_000, "n_z": 2000, "injections": 5_000_000, "batch": 128, "sets": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="precision_300ev")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--cpu-events", type=int, default=300)
    ap.add_argument("--cpu-lambdas", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-photo", action="store_true")
    ap.add_argument("--serve-chunk-gb", type=float, default=4.0,
                    help="the server's launch sequences of at most this much per-point scratch "
                         "(0: one per fused batch)")
    ap.add_argument("--no-population", action="store_true",
                    help="skip the incomplete-catalogue and smoothed-mass-edge steps")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the single-1D, Epanechnikov and binned kernels")
    ap.add_argument("--photo-one", action="store_true",
                    help="the photometric workload for the Xi0 = 1 truth only (default: the "
                         "three truths 0.6, 1.0, 1.8)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="first copy 1 GiB device to device (a kernel of known traffic "
                         "for calibrating the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build runs on a single MI355X and has no "
              f"multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2504_02034_amd import chimera

    if args.traffic_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    wl, cf, ev, inj, p, lam = build_inputs(args.workload, args.batch)
    B = lam.shape[0]
    ctx, es = chimera.context_from_prepared(p, inj, device=0, n_tab=8192)
    lam_t = torch.from_numpy(lam).cuda()
    res = {}
    for name, prec in (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32)):
        out, wall, lat, n, ms, evals = time_precision(ctx, es, lam_t, prec, args.steps,
                                                      args.warmup)
        avg_ms = ms / max(n, 1)
        per_launch = evals / max(n, 1)
        achieved = per_launch * FLOPS_PER_EVAL / (avg_ms * 1e-3) / 1e12
        res[name] = dict(out=out, wall=wall, lat=lat, avg_ms=avg_ms, evals=per_launch,
                         achieved=achieved)
        log(f"{name}: {wall / args.steps * 1e3:.2f} ms/step, event kernel {avg_ms:.2f} ms, "
            f"{per_launch:.3e} evals/launch, {achieved:.2f} TFLOP/s")
    l32, l64 = res["fp32"]["out"], res["fp64"]["out"]
    fin = np.isfinite(l64) & np.isfinite(l32)
    dmax = float(np.max(np.abs(l32[fin] - l64[fin]))) if fin.any() else None
    same_mask = bool(np.array_equal(np.isfinite(l32), np.isfinite(l64)))

    def roof(name):
        r = res[name]
        kern = "chimera::k_event_smooth" + name[2:]
        return {"bound": "alu", "achieved": round(r["achieved"], 3), "peak": PEAK_TFLOPS[name],
                "unit": "TFLOP/s", "frac": round(r["achieved"] / PEAK_TFLOPS[name], 4),
                "traffic": measured_traffic(kern, wl.name),
                "kernel": "k_event_smooth" + name[2:],
                "kernel_ms": round(r["avg_ms"], 4), "evals_per_launch": int(r["evals"]),
                "flops_per_eval": FLOPS_PER_EVAL,
                "frac_of_unpacked_peak": round(r["achieved"] / PEAK_TFLOPS_UNPACKED[name], 4),
                "counters": measured_counters(kern, wl.name)}

    k = args.steps
    w32 = res["fp32"]["wall"]
    line = {
        "metric": "lnL evals/s at 300 ev x 5k samples (FP32 vs FP64), p50/p99 latency, |dlnL|",
        "value": round(B * k / w32, 2),
        "unit": "lnL evals/s",
        "n_gpus": 1, "steps": k, "warmup": args.warmup,
        "ms_per_step": round(w32 / k * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "events": wl.n_events, "samples_per_event": wl.n_samples,
                   "galaxies": wl.n_galaxies, "nside": wl.nside, "n_z": wl.n_z,
                   "injections": wl.n_inj, "batch": B},
        "latency_ms": {"p50": round(pct(res["fp32"]["lat"], 50), 4),
                       "p99": round(pct(res["fp32"]["lat"], 99), 4)},
        "fp64": {"value": round(B * k / res["fp64"]["wall"], 2),
                 "ms_per_step": round(res["fp64"]["wall"] / k * 1e3, 4),
                 "latency_ms": {"p50": round(pct(res["fp64"]["lat"], 50), 4),
                                "p99": round(pct(res["fp64"]["lat"], 99), 4)}},
        "speedup_fp32_over_fp64": round(res["fp64"]["wall"] / w32, 3),
        "abs_dlnL_fp32_vs_fp64": {"max": dmax, "same_finite_mask": same_mask,
                                  "finite_points": int(fin.sum())},
        "roofline": roof("fp32"),
        "roofline_fp64": roof("fp64"),
    }
    if not args.no_grad:
        from paper_2504_02034_amd import synth
        lam_g = torch.from_numpy(synth.make_lambdas(synth.WORKLOADS["grad_300ev"])).cuda()
        g = {"batch": int(lam_g.shape[0]), "params": 12}
        for name, prec in (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32)):
            sec = time_grad(ctx, es, lam_g, prec, 3)
            g[name] = {"ms": round(sec * 1e3, 3), "evals_per_s": round(lam_g.shape[0] / sec, 1),
                       "over_forward": round(sec / (res[name]["wall"] / k * lam_g.shape[0] / B), 2)}
            log(f"grad {name}: {sec * 1e3:.2f} ms for {lam_g.shape[0]} lambda")
        g.update(grad_checks(ctx, es, lam_g))
        # the same points with the Epanechnikov kernel, and on 16-bin data sets
        for label, shape, nbins in (("epanechnikov", chimera.CHIMERA_KDE_EPANECHNIKOV, 0),
                                    ("gaussian_16_bins", chimera.CHIMERA_KDE_GAUSSIAN, 16)):
            ctx.set_event_kde(es, shape, nbins)
            try:
                ge = {}
                for name, prec in (("fp64", chimera.CHIMERA_FP64), ("fp32", chimera.CHIMERA_FP32)):
                    sec = time_grad(ctx, es, lam_g, prec, 3)
                    ge[name] = {"ms": round(sec * 1e3, 3),
                                "over_gaussian": round(sec * 1e3 / g[name]["ms"], 3)}
                    log(f"grad {label} {name}: {sec * 1e3:.2f} ms for {lam_g.shape[0]} lambda")
                g[label] = ge
            finally:
                ctx.set_event_kde(es)
        line["grad"] = g
    if not args.no_variants:
        line["kernel_variants"] = variants_bench(ctx, es, p, ev, lam_t, res, args.steps,
                                                 args.warmup)
    if not args.no_population:
        line["population_variants"] = population_bench(ctx, es, wl, p, lam_t, res, args.steps,
                                                       args.warmup)
    ctx.close()
    if not args.no_serve:
        line["serving"] = serve_bench(wl, cf, inj, chunk_gb=args.serve_chunk_gb)
    if not args.no_photo:
        log("photometric workload")
        line["photometric"] = photo_bench((1.0,) if args.photo_one else (0.6, 1.0, 1.8))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (cpu_baseline)")
        fin_idx = np.flatnonzero(np.isfinite(res["fp64"]["out"]))[:args.cpu_lambdas]
        if fin_idx.size == 0:
            fin_idx = np.arange(min(args.cpu_lambdas, B))
        line["cpu_baseline"] = cpu_baseline(wl, cf, ev, inj, lam[fin_idx], args.cpu_events)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
