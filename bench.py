#!/usr/bin/env python3
"""Benchmark of the Hough-transform fill + peak search on one MI355X.

One step = one event of the paper-shaped workload (5000 hits, 4 theta x 16 phi x 1024 A x 1024 B
uint32 vote matrix, threshold 9) through the whole path: per-hit prep and bucketing, the fill
(which writes every cell of the 256 MiB matrix), the peak search, and the return of the peak
list to pinned host memory. Inputs are resident in HBM when the timed region starts. Prints one
JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s + Gvotes/s on 1 MI355X; p50/p99 event latency, served vs plain"
HBM_PEAK_GBS = 8000.0
# Launch shape of the timed loop (rows, group_tiles, cand_cap, nt_store, tiles_per_block; 0 or -1
# for the library's default of a field), measured fastest on MI355X with the matrices cycled;
# the committed profiles are taken at it.
PINNED_TUNING = "4,16,0,1,1"
# Launch shapes the batch autotuner picks for the batched (workload 2) and stress (workload 4)
# batches on MI355X; --only pins them, so that a profiled run times no search.
BATCH_TUNING = {"batched": "4,16,256,1,2", "stress": "4,16,256,1,8"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def cpu_baseline(spec, workload, seconds):
    """The oracle on a bounded sample of the same workload: one thread (per-event latency), then
    one oracle thread per event on the host cores given to this process (up to 16), each with
    its own matrix (events are independent). ctypes drops the GIL inside the oracle's C calls."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle
    from paper_1507_03074_amd import synth
    g = oracle.OracleGrid(*spec.as_tuple())
    oracle.check_grid(g)  # loads the library once, before any thread starts

    def one(seed, buf):
        ev = synth.make_event(workload, seed)
        t0 = time.perf_counter()
        M, v = oracle.fill(g, ev.x, ev.y, ev.z, out=buf)
        t1 = time.perf_counter()
        oracle.peaks(g, M)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, v

    buf = np.empty(spec.shape, np.uint32)
    single, t0 = [], time.perf_counter()
    while len(single) < 3 or (time.perf_counter() - t0 < seconds / 2 and len(single) < 100):
        single.append(one(1000 + len(single), buf))
    t_fill = sum(r[0] for r in single) / len(single)
    t_peaks = sum(r[1] for r in single) / len(single)
    n_thr = max(1, min(16, len(os.sched_getaffinity(0))))
    bufs = [np.empty(spec.shape, np.uint32) for _ in range(n_thr)]
    deadline = time.perf_counter() + seconds / 2

    def worker(i):
        done, k = 0, 0
        while done < 2 or time.perf_counter() < deadline:
            one(2000 + i * 1000 + k, bufs[i])
            done += 1
            k += 1
        return done

    t0 = time.perf_counter()
    with ThreadPoolExecutor(n_thr) as pool:
        counts = list(pool.map(worker, range(n_thr)))
    t_all = time.perf_counter() - t0
    return dict(value=round(sum(counts) / t_all, 3), unit="events/s", cores=n_thr, kind="oracle",
                sample="workload 1 events (5000 hits, 4x16x1024x1024), fill + peaks: %d events on %d "
                       "threads in %.1f s; single thread %d events" % (sum(counts), n_thr, t_all, len(single)),
                single_thread={"events_per_s": round(1.0 / (t_fill + t_peaks), 3),
                               "fill_ms": round(t_fill * 1e3, 2), "peaks_ms": round(t_peaks * 1e3, 2)},
                host_cpu=host_cpu_model()), single


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def measure_peaks(B, torch, acc_bytes, big_bytes=2 << 30):
    """Ceilings measured in the same run (one launch each, timed with events on this stream).
    Streams run over a buffer far larger than the 256 MiB last-level MALL (the true HBM rate)
    and over a buffer of the vote matrix's size (what the fill itself sees)."""
    stream = torch.cuda.current_stream()
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    L = B.lib()
    sp = ctypes_stream(stream)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / 1e3 / reps

    def streams(nbytes):
        buf = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
        buf2 = torch.empty_like(buf)
        t_wm = [timed(lambda m=m: L.ht_bench_hbm_write(buf.data_ptr(), nbytes, m, sp)) for m in (0, 1, 2, 3, 4)]
        t_r = timed(lambda: L.ht_bench_hbm_read(buf.data_ptr(), nbytes, sink.data_ptr(), sp))
        t_c = timed(lambda: L.ht_bench_copy(buf2.data_ptr(), buf.data_ptr(), nbytes, sp))
        del buf, buf2
        torch.cuda.empty_cache()
        return {"write_GBs": round(nbytes / min(t_wm) / 1e9, 1),
                "write_GBs_by_mode": {"nontemporal16": round(nbytes / t_wm[0] / 1e9, 1),
                                      "store16": round(nbytes / t_wm[1] / 1e9, 1),
                                      "store4": round(nbytes / t_wm[2] / 1e9, 1),
                                      "tiles_nontemporal16": round(nbytes / t_wm[3] / 1e9, 1),
                                      "tiles_store16": round(nbytes / t_wm[4] / 1e9, 1)},
                "read_GBs": round(nbytes / t_r / 1e9, 1),
                "copy_GBs": round(2 * nbytes / t_c / 1e9, 1),
                "buffer_MiB": nbytes >> 20}

    big = streams(big_bytes)
    mat = streams(acc_bytes)
    buf = torch.empty(acc_bytes // 4, dtype=torch.int32, device="cuda")
    n_ops = 1 << 28
    t_a = timed(lambda: L.ht_bench_atomic_rand(buf.data_ptr(), buf.numel(), n_ops, sp), reps=3)
    small = 1 << 20  # 4 MiB: an L2-resident target
    t_al = timed(lambda: L.ht_bench_atomic_rand(buf.data_ptr(), small, n_ops, sp), reps=3)
    blocks, iters = 256 * 16, 4096
    t_l = timed(lambda: L.ht_bench_lds_atomic(blocks, iters, sink.data_ptr(), sp), reps=3)
    del buf
    torch.cuda.empty_cache()
    return {"hbm_write_GBs": big["write_GBs"], "hbm_read_GBs": big["read_GBs"],
            "copy_GBs": big["copy_GBs"], "large_buffer": big, "matrix_sized_buffer": mat,
            "atomic_rand_Gops": round(n_ops / t_a / 1e9, 2),
            "atomic_l2_Gops": round(n_ops / t_al / 1e9, 2),
            "lds_atomic_Gops": round(blocks * 256 * iters / t_l / 1e9, 1)}


def bench_batched(B, torch, synth, workload, n_events, reps, capacity, tune_batch=False):
    """One ht_fill_peaks_batch call (a captured graph) over n_events events of the workload;
    with tune_batch, the launch shape comes from the autotuner run on another batch of the same
    workload (events n_events .. 2 n_events - 1, kept apart from the timed ones), and the grid's
    previous shape is restored afterwards."""
    spec = synth.WORKLOADS[workload].grid
    evs = [synth.make_event(workload, e) for e in range(n_events)]
    tuned = None
    if tune_batch:
        from paper_1507_03074_amd import tune
        before = B.ht_get_tuning(spec)
        tevs = [synth.make_event(workload, n_events + e) for e in range(n_events)]
        rep = tune.autotune_batch(spec, [(e.x, e.y, e.z) for e in tevs], capacity=capacity)
        del tevs
        tuned = {"best": rep["best"], "default_ms_per_batch": round(rep["default_ms_per_batch"], 3),
                 "candidates": len(rep["candidates"]),
                 "events": "workload %d, seeds %d-%d" % (workload, n_events, 2 * n_events - 1)}
    xs = np.concatenate([e.x for e in evs])
    ys = np.concatenate([e.y for e in evs])
    zs = np.concatenate([e.z for e in evs])
    x, y, z = B.hits_to_device(xs, ys, zs)
    events, off = [], 0
    for i, e in enumerate(evs):
        events.append(B.Event(off, e.n, i * capacity, capacity))
        off += e.n
    acc = B.new_acc(spec, n_events)
    out = torch.empty((n_events * capacity, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(n_events, dtype=torch.int64, device="cuda")
    B.ht_fill_peaks_batch(spec, events, x, y, z, acc, out, nf)
    torch.cuda.synchronize()
    votes = int(acc.sum(dtype=torch.int64).item())
    # two untimed batches after the first (which captures the graph), so the timed ones start
    # from a running GPU
    for _ in range(2):
        B.ht_fill_peaks_batch(spec, events, x, y, z, acc, out, nf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        B.ht_fill_peaks_batch(spec, events, x, y, z, acc, out, nf)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res = {"workload": synth.WORKLOADS[workload].name, "events_per_batch": n_events,
           "hits_mean": round(float(np.mean([e.n for e in evs])), 1),
           "ms_per_batch": round(dt * 1e3, 3), "events_per_s": round(n_events / dt, 1),
           "gvotes_per_s": round(votes / dt / 1e9, 2),
           "hbm_write_GBs": round(4 * spec.n_cells * n_events / dt / 1e9, 1),
           "peaks_per_event": round(float(nf.float().mean().item()), 1),
           "max_peaks": int(nf.max().item()), "capacity": capacity,
           "tuning": B.ht_get_tuning(spec).as_dict(), "autotune": tuned}
    if tune_batch:
        B.ht_set_tuning(spec, before)
    del acc, out, x, y, z
    torch.cuda.empty_cache()
    return res


def bench_served(B, torch, synth, n_pool, n_warm, n_meas, rates, budget_gib, max_batch, n_streams,
                 serve_tuning=None):
    """Served vs plain on workload 3: the same Poisson arrival traces are replayed through the
    request loop (continuous batching over streams) and through one-at-a-time ht_fill_peaks.
    Both take each event's hits from host memory and deliver its peaks to host memory.
    serve_tuning (a tuning dict): the launch shape the server is created with (it keeps the shape
    it was created with); the plain path keeps the grid's current shape."""
    spec = synth.WORKLOADS[3].grid
    pool = [synth.make_event(3, e) for e in range(n_pool)]
    cap = 1 << 17
    res = {"workload": synth.WORKLOADS[3].name, "pool_events": n_pool,
           "hits_mean": round(float(np.mean([e.n for e in pool])), 1),
           "max_batch": max_batch, "n_streams": n_streams, "hbm_budget_GiB": budget_gib}

    # plain: one event at a time, synchronous. Like the request loop, it takes each event's hits
    # from host memory (here already in pinned buffers, x, y and z packed, one upload per event)
    # and has the peak list written to pinned host memory.
    host_pool = []
    for e in pool:
        hp = torch.empty(3 * e.n, dtype=torch.float32, pin_memory=True)
        hp[:e.n] = torch.from_numpy(np.ascontiguousarray(e.x, np.float32))
        hp[e.n:2 * e.n] = torch.from_numpy(np.ascontiguousarray(e.y, np.float32))
        hp[2 * e.n:] = torch.from_numpy(np.ascontiguousarray(e.z, np.float32))
        host_pool.append(hp)
    dev_hits = torch.empty(3 * max(e.n for e in pool), dtype=torch.float32, device="cuda")
    acc = B.new_acc(spec)
    h_out = torch.empty((cap, 2), dtype=torch.int32, pin_memory=True)
    h_nf = torch.zeros(1, dtype=torch.int64, pin_memory=True)
    stream = torch.cuda.current_stream()

    def plain_one(i):
        hp = host_pool[i % n_pool]
        n = hp.numel() // 3
        d = dev_hits[:3 * n]
        d.copy_(hp, non_blocking=True)
        B.ht_fill_peaks(spec, d[:n], d[n:2 * n], d[2 * n:], acc, h_out, cap, h_nf, stream)
        stream.synchronize()  # waits for the event, as a caller needing its result does

    for i in range(20):
        plain_one(i)
    t0 = time.perf_counter()
    for i in range(200):
        plain_one(i)
    plain_rate = 200 / (time.perf_counter() - t0)
    res["plain_saturation_events_per_s"] = round(plain_rate, 1)

    plain_tuning = B.ht_get_tuning(spec)
    if serve_tuning:
        B.ht_set_tuning(spec, B.Tuning(**serve_tuning))
    srv_ctx = B.Server(spec, budget_gib << 30, peak_capacity=cap, max_hits=40000, max_batch=max_batch,
                       n_streams=n_streams, queue_depth=1024)
    B.ht_set_tuning(spec, plain_tuning)
    res["serve_tuning"] = serve_tuning
    res["plain_tuning"] = plain_tuning.as_dict()
    with srv_ctx as srv:
        def run_trace(arrivals):
            n = len(arrivals)
            lat, pending, i, done = [], {}, 0, 0
            order = []
            t_base = time.perf_counter()
            while done < n:
                now = time.perf_counter() - t_base
                if i < n and now >= arrivals[i]:
                    ev = pool[i % n_pool]
                    t = srv.submit(ev.x, ev.y, ev.z)
                    if t is not None:
                        pending[t] = i
                        order.append(t)
                        i += 1
                        continue
                # collect finished requests (oldest first)
                progressed = False
                for t in list(order[:64]):
                    r = srv.poll(t)
                    if r is None:
                        continue
                    _, _, n_found, tm = r
                    lat.append((pending.pop(t), tm.t_done - tm.t_submit, tm))
                    order.remove(t)
                    done += 1
                    progressed = True
                if not progressed and i >= n:
                    time.sleep(20e-6)
            t_end = time.perf_counter() - t_base
            lat.sort()
            return lat, t_end

        # saturation: everything arrives at once, after one untimed pass of n_warm events (the
        # server's first batches touch its memory for the first time)
        run_trace(np.zeros(n_warm))
        lat, t_end = run_trace(np.zeros(n_warm + n_meas))
        sat = (n_warm + n_meas) / t_end
        res["served_saturation_events_per_s"] = round(sat, 1)
        res["rates"] = []
        for frac in rates:
            rate = frac * sat
            arr = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, n_warm + n_meas))
            lat, t_end = run_trace(arr)
            served = np.array([l for _, l, _ in lat[n_warm:]]) * 1e3
            tms = [tm for _, _, tm in lat[n_warm:]]
            parts = {"queue": [t.t_admit - t.t_submit for t in tms],
                     "admit_to_launch": [t.t_launch - t.t_admit for t in tms],
                     "launch_to_done": [t.t_done - t.t_launch for t in tms]}
            # plain replay of the same trace: a FIFO single server
            t_base = time.perf_counter()
            plain = []
            for i, a in enumerate(arr):
                while time.perf_counter() - t_base < a:
                    pass
                plain_one(i)
                if i >= n_warm:
                    plain.append((time.perf_counter() - t_base - a) * 1e3)
            plain = np.array(plain)
            res["rates"].append({
                "offered_events_per_s": round(rate, 1), "fraction_of_served_saturation": frac,
                "served_p50_ms": round(float(np.percentile(served, 50)), 3),
                "served_p99_ms": round(float(np.percentile(served, 99)), 3),
                "served_events_per_s": round((n_warm + n_meas) / t_end, 1),
                "plain_p50_ms": round(float(np.percentile(plain, 50)), 3),
                "plain_p99_ms": round(float(np.percentile(plain, 99)), 3),
                "served_parts_p50_p99_ms": {k: [round(float(np.percentile(v, 50)) * 1e3, 3),
                                                round(float(np.percentile(v, 99)) * 1e3, 3)]
                                            for k, v in parts.items()}})
    del acc, dev_hits, host_pool
    torch.cuda.empty_cache()
    return res


def bench_transfers(B, torch, synth, spec, sizes=(500, 1000, 2000, 4000, 8000), reps=20):
    """Where the paper's time went (its Fig. 3g: device-to-host transfer dominated): copy costs
    of the full vote matrix versus the peak list only, hit uploads, and a hit-count sweep of the
    stage times."""
    stream = torch.cuda.current_stream()
    acc = B.new_acc(spec)
    cap = 1 << 14
    out, nf = B.new_peaks(cap)
    res = {}

    def tcopy(dst, src, n=5):
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    host_pinned = torch.empty(acc.shape, dtype=torch.int32, pin_memory=True)
    host_page = torch.empty(acc.shape, dtype=torch.int32)
    res["matrix_d2h_pinned_ms"] = round(tcopy(host_pinned, acc) * 1e3, 3)
    res["matrix_d2h_pageable_ms"] = round(tcopy(host_page, acc, 2) * 1e3, 3)
    res["matrix_bytes"] = acc.numel() * 4
    del host_pinned, host_page
    ev = synth.make_event(1, 0)
    x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
    B.ht_fill_peaks(spec, x, y, z, acc, out, cap, nf)
    n = int(nf.item())
    hp = torch.empty((cap, 2), dtype=torch.int32, pin_memory=True)
    res["peaks_d2h_us"] = round(tcopy(hp[:n], out[:n], 50) * 1e6, 2)
    res["peaks_bytes"] = n * 8
    hx = torch.from_numpy(np.ascontiguousarray(ev.x))
    hxp = hx.pin_memory()
    res["hits_h2d_pinned_us"] = round(3 * tcopy(x, hxp, 50) * 1e6, 2)
    res["hits_h2d_pageable_us"] = round(3 * tcopy(x, hx, 50) * 1e6, 2)
    sweep = []
    for nh in sizes:
        nt, nn = synth.hits_split(nh)
        e = synth.make_hits(np.random.default_rng(9000 + nh), nt, nn)
        xd, yd, zd = B.hits_to_device(e.x, e.y, e.z)
        for _ in range(3):
            B.ht_fill_peaks(spec, xd, yd, zd, acc, out, cap, nf)
        torch.cuda.synchronize()
        for st in ("prep", "fill", "peaks"):
            B.ht_profile_read(st, reset=True)
        B.ht_profile_enable(True)
        for _ in range(reps):
            B.ht_fill_peaks(spec, xd, yd, zd, acc, out, cap, nf)
        torch.cuda.synchronize()
        B.ht_profile_enable(False)
        row = {"hits": nh}
        for st in ("prep", "fill", "peaks"):
            ms, c = B.ht_profile_read(st)
            row[st + "_us"] = round(ms / max(c, 1) * 1e3, 2)
        B.ht_profile_read("fill", reset=True)
        k = int(nf.item())
        row["peaks"] = k
        row["peaks_d2h_us"] = round(tcopy(hp[:max(k, 1)], out[:max(k, 1)], 20) * 1e6, 2)
        sweep.append(row)
    res["hit_sweep"] = sweep
    del acc, out
    torch.cuda.empty_cache()
    return res


# the sources whose text defines the fill kernels (the template, its instantiations and the
# structures it reads)
KERNEL_SOURCES = ("ht_internal.h", "ht_device.h", "ht_fill_rows.hip")


def kernel_sources_sha256():
    """SHA-256 over the fill kernels' sources, in a fixed order: counters taken on other sources
    no longer describe the kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1507_03074_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counter_traffic(tuning: dict):
    """HBM bytes per fill launch from the committed FETCH_SIZE / WRITE_SIZE counter summary
    (each counter scaled by what it reads for a copy of known size), or None when the summary
    was taken on other kernel sources or with another fill shape (A rows per tile, store kind,
    tiles per workgroup)."""
    import re
    path = os.path.join(ROOT, "profiles", "k_fill_paper-event_counters.md")
    try:
        text = open(path).read()
        recs = [json.loads(m) for m in re.findall(r"```json\n(.*?)\n```", text, re.S)]
        sha = kernel_sources_sha256()
    except (OSError, ValueError):
        return None
    shape = [tuning[f] for f in ("rows", "nt_store", "tiles_per_block")]
    for rec in recs:
        if rec.get("kernels_source_sha256") != sha or rec.get("fill_shape") != shape:
            continue
        for name, v in rec["per_launch"].items():
            if name.startswith("k_fill<%d," % tuning["rows"]):
                return v["traffic_bytes"]
    return None


def bench_two_streams(B, torch, spec, dev_hits, h_out, h_nf, cap, steps):
    """The same per-event call issued alternately on two streams with two matrices, so that the
    short prep and peak kernels of one event overlap the other event's fill (each stream has its
    own library workspace). Not the headline number, which is the plain one-stream loop."""
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    accs = [B.new_acc(spec), B.new_acc(spec)]
    n = len(dev_hits)

    def step(k):
        j = k & 1
        i = k % n
        x, y, z = dev_hits[i]
        B.ht_fill_peaks(spec, x, y, z, accs[j], h_out[i], cap, h_nf[i:i + 1], streams[j])

    for k in range(40):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    del accs
    torch.cuda.empty_cache()
    return {"ms_per_event": round(dt * 1e3, 4), "events_per_s": round(1.0 / dt, 1)}


def bench_sectors(B, torch, synth, evs, dev_hits, steps):
    """The sector variant (paper section 4) on the paper-shaped events: four phi sectors, one
    M_H(A, B, theta) each (4 x 4 x 1024 x 1024, 64 MiB), through the plain per-event path, and
    its track finding next to the 4-D transform's (16 widened phi cells) on the same events."""
    from paper_1507_03074_amd import physics
    spec4 = synth.WORKLOADS[1].grid
    specS = synth.GridSpec(4, 4, 1024, 1024, threshold=spec4.threshold, phi_sectors=True)
    stream = torch.cuda.current_stream()
    cap = 4096
    acc = B.new_acc(specS)
    out, nf = B.new_peaks(cap)
    n = len(dev_hits)
    for k in range(20):
        x, y, z = dev_hits[k % n]
        B.ht_fill_peaks(specS, x, y, z, acc, out, cap, nf, stream)
    torch.cuda.synchronize()
    B.ht_profile_read("fill", reset=True)
    B.ht_profile_enable(2)
    t0 = time.perf_counter()
    for k in range(steps):
        x, y, z = dev_hits[k % n]
        B.ht_fill_peaks(specS, x, y, z, acc, out, cap, nf, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    B.ht_profile_enable(0)
    fill_ms, fill_n = B.ht_profile_read("fill", reset=True)
    res = {"grid": list(specS.shape), "matrix_MiB": specS.n_cells * 4 >> 20,
           "ms_per_event": round(dt * 1e3, 4), "events_per_s": round(1.0 / dt, 1),
           "fill_us": round(fill_ms / max(fill_n, 1) * 1e3, 2)}
    # track finding: sectors against the 4-D transform on the same events
    acc4 = B.new_acc(spec4)
    out4, nf4 = B.new_peaks(cap)
    cmp = {"events": 0, "in_acceptance": 0, "found_4d": 0, "found_sectors": 0,
           "lost_in_sectors": 0, "lost_in_sectors_crossing_a_sector_edge": 0,
           "gained_in_sectors": 0, "peaks_4d": 0, "peaks_sectors": 0}
    for i in range(min(8, n)):
        x, y, z = dev_hits[i]
        B.ht_fill_peaks(spec4, x, y, z, acc4, out4, cap, nf4, stream)
        B.ht_fill_peaks(specS, x, y, z, acc, out, cap, nf, stream)
        t4 = B.tracks_to_host(B.ht_readout(spec4, out4, nf4, cap), nf4, cap)
        tS = B.tracks_to_host(B.ht_readout(specS, out, nf, cap), nf, cap)
        e4 = physics.evaluate(spec4, t4, evs[i])
        eS = physics.evaluate(specS, tS, evs[i])
        f4, fS = set(e4["found_ids"]), set(eS["found_ids"])
        ev = evs[i]
        crossing = 0
        for k in f4 - fS:
            own = ev.track_of_hit == k
            ph = np.mod(np.arctan2(ev.y[own].astype(np.float64), ev.x[own].astype(np.float64)), 2 * np.pi)
            crossing += len(set(np.floor(ph / (np.pi / 2)).astype(int).tolist())) > 1
        cmp["events"] += 1
        cmp["in_acceptance"] += e4["in_acceptance"]
        cmp["found_4d"] += len(f4)
        cmp["found_sectors"] += len(fS)
        cmp["lost_in_sectors"] += len(f4 - fS)
        cmp["lost_in_sectors_crossing_a_sector_edge"] += crossing
        cmp["gained_in_sectors"] += len(fS - f4)
        cmp["peaks_4d"] += e4["peaks"]
        cmp["peaks_sectors"] += eS["peaks"]
    cmp["efficiency_4d"] = round(cmp["found_4d"] / max(1, cmp["in_acceptance"]), 4)
    cmp["efficiency_sectors"] = round(cmp["found_sectors"] / max(1, cmp["in_acceptance"]), 4)
    res["vs_4d"] = cmp
    del acc, acc4
    torch.cuda.empty_cache()
    return res


def ctypes_stream(stream):
    import ctypes
    return ctypes.c_void_p(stream.cuda_stream)


def bench_crowded(B, torch, synth, steps, tuning=None):
    """Stage times on the smallest, median and largest of 40 events of workload 3 (lognormal
    5k-40k hits on the paper grid), at the given launch shape or the library's default. The
    largest event pools 2.6M candidates, so its peak stage runs the many-candidate test."""
    spec = synth.WORKLOADS[3].grid
    if tuning:
        B.ht_set_tuning(spec, B.Tuning(*[int(v) for v in tuning.split(",")]))
    evs = sorted((synth.make_event(3, e) for e in range(40)), key=lambda e: e.n)
    cap = 1 << 19
    acc = B.new_acc(spec)
    out, nf = B.new_peaks(cap)
    res = {"workload": synth.WORKLOADS[3].name, "tuning": B.ht_get_tuning(spec).as_dict(), "events": []}
    for ev in (evs[0], evs[len(evs) // 2], evs[-1]):
        x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
        for _ in range(5):
            B.ht_fill_peaks(spec, x, y, z, acc, out, cap, nf)
        torch.cuda.synchronize()
        B.ht_profile_read("fill", reset=True)
        B.ht_profile_enable(1)
        for _ in range(steps):
            B.ht_fill_peaks(spec, x, y, z, acc, out, cap, nf)
        torch.cuda.synchronize()
        B.ht_profile_enable(0)
        us = {st: round(B.ht_profile_read(st)[0] / steps * 1e3, 1) for st in ("prep", "fill", "peaks")}
        B.ht_profile_read("fill", reset=True)
        res["events"].append({"hits": ev.n, "peaks": int(nf.item()), "stage_us": us})
    if tuning:
        B.ht_set_tuning(spec)
    return res


def bench_crossover(B, torch, synth, steps):
    """The whole fused call (prep, fill, peak search) on served-stream events of 6k-40k hits
    (workload 3, paper grid), once with every event's peaks from the candidate pool and once
    from the stencil over the matrix: where the library's default threshold between the two
    comes from. Peak counts must agree."""
    import os
    spec = synth.WORKLOADS[3].grid
    sizes = [synth.event_size(3, e) for e in range(300)]
    cap = 1 << 19
    acc = B.new_acc(spec)
    out, nf = B.new_peaks(cap)
    saved = os.environ.get("HT_DENSE_HITS")
    rows = []
    for want in (6000, 9000, 12000, 15000, 18000, 22000, 26000, 30000, 35000, 40000):
        e = int(np.argmin([abs(n - want) for n in sizes]))
        ev = synth.make_event(3, e)
        x, y, z = B.hits_to_device(ev.x, ev.y, ev.z)
        row = {"hits": ev.n}
        for mode, val in (("pool", "-1"), ("stencil", "1")):
            os.environ["HT_DENSE_HITS"] = val
            for _ in range(3):
                B.ht_fill_peaks(spec, x, y, z, acc, out, cap, nf)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                B.ht_fill_peaks(spec, x, y, z, acc, out, cap, nf)
            torch.cuda.synchronize()
            row[mode + "_us"] = round((time.perf_counter() - t0) / steps * 1e6, 1)
            row[mode + "_peaks"] = int(nf.item())
        assert row["pool_peaks"] == row["stencil_peaks"]
        rows.append(row)
    if saved is None:
        os.environ.pop("HT_DENSE_HITS", None)
    else:
        os.environ["HT_DENSE_HITS"] = saved
    return {"workload": synth.WORKLOADS[3].name, "default_dense_hits": B.ht_get_tuning(spec).dense_hits,
            "events": rows}


def pinned_tuning(text):
    return [int(v) for v in text.split(",")]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--events", type=int, default=16, help="distinct resident events cycled")
    ap.add_argument("--matrices", type=int, default=16,
                    help="vote matrices cycled by the timed loop (16 x 256 MiB = 4 GiB, far past "
                         "the 256 MB last-level cache, so every matrix write reaches HBM)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="main line only (no extra workloads)")
    ap.add_argument("--tuning", default=PINNED_TUNING,
                    help="rows,group_tiles,cand_cap,nt_store,tiles_per_block of the timed loop "
                         "(default: the shape pinned here, which the committed profiles use)")
    ap.add_argument("--autotune", action="store_true",
                    help="search the launch shape on four separate events (cycling --matrices "
                         "matrices) instead of using --tuning")
    ap.add_argument("--counters", action="store_true",
                    help="for hardware-counter runs: a 256 MiB copy (the byte-counter reference) "
                         "three times, then --steps steps of the timed loop untimed, then three "
                         "plain atomic fills; prints one line")
    ap.add_argument("--crowded", action="store_true",
                    help="stage times on small, median and crowded events of the served stream "
                         "(workload 3) at the --tuning shape or the default; prints one line")
    ap.add_argument("--crossover", action="store_true",
                    help="time the fused call on served-stream events of 6k-40k hits with the "
                         "candidate pool and with the stencil peak search; prints one line")
    ap.add_argument("--only", choices=("batched", "stress", "served"),
                    help="one workload only, for profiles: the batched workload 2 (100 events, "
                         "one graph launch) or the stress workload 4 (16 events) at the launch "
                         "shape the batch autotuner picks, --steps capped at 10 batches; or the "
                         "served workload 3 at its saturation rate (1200 events); prints one "
                         "line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path. Events are "
              "independent, so several GPUs would each run their own events (or request loop) "
              "with no collective between them.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1507_03074_amd import binding as B
    from paper_1507_03074_amd import synth

    from paper_1507_03074_amd import build as hbuild
    hbuild.ensure_built()  # a missing or stale library is rebuilt, never measured
    torch.cuda.set_device(0)
    if args.crowded:
        tuning = None if args.tuning == PINNED_TUNING else args.tuning
        print(json.dumps({"crowded": bench_crowded(B, torch, synth, min(args.steps, 50), tuning)}),
              flush=True)
        return
    if args.crossover:
        print(json.dumps({"crossover": bench_crossover(B, torch, synth, min(args.steps, 20))}), flush=True)
        return
    if args.only in ("batched", "stress"):
        wl, n_ev, cap_b = (2, 100, 1 << 13) if args.only == "batched" else (4, 16, 1 << 21)
        B.ht_set_tuning(synth.WORKLOADS[wl].grid, B.Tuning(*pinned_tuning(BATCH_TUNING[args.only])))
        res = bench_batched(B, torch, synth, wl, n_ev, min(args.steps, 10), cap_b)
        print(json.dumps({args.only: res}), flush=True)
        return
    if args.only == "served":
        B.ht_set_tuning(synth.WORKLOADS[3].grid, B.Tuning(*pinned_tuning(args.tuning)))
        res = bench_served(B, torch, synth, n_pool=128, n_warm=200, n_meas=1000, rates=(1.0,),
                           budget_gib=24, max_batch=8, n_streams=2)
        print(json.dumps({"served": res}), flush=True)
        return
    workload = 1
    spec = synth.WORKLOADS[workload].grid
    cap = 4096
    log("generating %d events of workload %d" % (args.events, workload))
    evs = [synth.make_event(workload, e) for e in range(args.events)]
    dev_hits = [B.hits_to_device(e.x, e.y, e.z) for e in evs]
    mats = [B.new_acc(spec) for _ in range(max(1, args.matrices))]
    acc = mats[0]
    out = torch.empty((args.events, cap, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(args.events, dtype=torch.int64, device="cuda")
    h_out = torch.empty((args.events, cap, 2), dtype=torch.int32, pin_memory=True)
    h_nf = torch.zeros(args.events, dtype=torch.int64, pin_memory=True)
    stream = torch.cuda.current_stream()

    def step(k, ms=mats):
        # event k % E into matrix k % M; the peak kernel writes the peak list and its count
        # straight into pinned host memory
        i = k % args.events
        x, y, z = dev_hits[i]
        B.ht_fill_peaks(spec, x, y, z, ms[k % len(ms)], h_out[i], cap, h_nf[i:i + 1], stream)

    if args.counters:
        B.ht_set_tuning(spec, B.Tuning(*pinned_tuning(args.tuning)))
        copy_bytes = 256 << 20
        src = torch.zeros(copy_bytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            B.check(B.lib().ht_bench_copy(dst.data_ptr(), src.data_ptr(), copy_bytes, ctypes_stream(stream)))
        torch.cuda.synchronize()
        for k in range(args.steps):
            step(k)
        torch.cuda.synchronize()
        # then the plain atomic fill (one global atomicAdd per vote) on the first three events
        for i in range(3):
            x, y, z = dev_hits[i % args.events]
            B.ht_fill(spec, x, y, z, acc, stream, atomic=True)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "copy_bytes": copy_bytes, "copies": 3,
                          "steps": args.steps, "matrices": len(mats), "atomic_fills": 3,
                          "tuning": B.ht_get_tuning(spec).as_dict()}), flush=True)
        return

    # launch shape: the pinned one (the committed profiles are taken at it), or a search on
    # events kept apart from the timed set (every candidate gated on bit-exact results)
    if args.autotune:
        from paper_1507_03074_amd import tune
        log("autotuning the launch shape")
        tevs = [synth.make_event(workload, 100 + e) for e in range(4)]
        rep = tune.autotune(spec, [(e.x, e.y, e.z) for e in tevs], reps=30, n_acc=min(len(mats), 8))
        tuned = {"best": rep["best"], "default_us_per_event": round(rep["default_us_per_event"], 2),
                 "candidates": len(rep["candidates"]), "events": "workload 1, seeds 100-103"}
    else:
        B.ht_set_tuning(spec, B.Tuning(*pinned_tuning(args.tuning)))
        tuned = {"pinned": args.tuning}

    # votes per event (the matrix sum; equal to the oracle's count by the parity tests)
    votes = []
    for i in range(args.events):
        x, y, z = dev_hits[i]
        B.ht_fill(spec, x, y, z, acc)
        votes.append(int(acc.sum(dtype=torch.int64).item()))

    def timed_loop(ms, steps):
        """K steps between two device synchronisations; the library records a HIP event pair
        around each fill launch on `stream` (the fill kernel's own duration, for the roofline);
        nothing else is timed inside it."""
        for k in range(args.warmup):
            step(k, ms)
        torch.cuda.synchronize()
        B.ht_profile_read("fill", reset=True)
        B.ht_profile_enable(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(k, ms)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.ht_profile_enable(0)
        f_ms, f_n = B.ht_profile_read("fill", reset=True)
        return t1 - t0, f_ms / 1000.0 / max(f_n, 1)

    # the headline: every event's matrix its own (4 GiB in all), so the writes reach HBM
    elapsed, fill_avg_s = timed_loop(mats, args.steps)
    ms_per_step = 1000.0 * elapsed / args.steps
    ev_per_s = args.steps / elapsed
    total_votes = sum(votes[k % args.events] for k in range(args.steps))
    nfound = h_nf.numpy().copy()
    # beside it: one matrix rewritten every step, which stays in the 256 MB last-level cache
    elapsed1, fill_avg1_s = timed_loop([acc], args.steps)

    # outside the timed region: the same loop with events around every stage (breakdown), and
    # with no events at all (the cost of the timing events themselves)
    n_extra = min(args.steps, 200)
    B.ht_profile_enable(1)
    for k in range(n_extra):
        step(k)
    torch.cuda.synchronize()
    B.ht_profile_enable(0)
    stage = {}
    for st in ("prep", "fill", "peaks"):
        ms, n = B.ht_profile_read(st)
        stage[st] = round(ms / max(n, 1), 4)
    B.ht_profile_read("fill", reset=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(n_extra):
        step(k)
    torch.cuda.synchronize()
    t3 = time.perf_counter()

    cells = spec.n_cells
    t = B.ht_tiling(spec)
    # (hit, cell) records per event: the fill reads each bucketed record (16 B)
    entries = []
    for x, y, z in dev_hits:
        info, _, _ = B.ht_debug_hit_values(spec, x, y, z)
        entries.append(int(info[:, 3].sum().item()))
    # algorithmic bytes of one fill launch: the matrix written once (4 B per cell) plus each
    # bucketed (hit, cell) record read once (16 B)
    hit_entries = float(np.mean(entries))
    alg_bytes = 4.0 * cells + 16.0 * hit_entries
    achieved = alg_bytes / fill_avg_s / 1e9
    achieved1 = alg_bytes / fill_avg1_s / 1e9
    tuning_now = B.ht_get_tuning(spec).as_dict()
    line = {
        "metric": METRIC,
        "value": round(ev_per_s, 2),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": synth.WORKLOADS[workload].name, "hits_per_event": 5000,
                   "grid": list(spec.shape), "threshold": spec.threshold,
                   "path": "ht_fill_peaks (fused), peak list written to pinned host memory",
                   "tile_rows": t["rows"], "resident_events": args.events,
                   "matrices_cycled": len(mats), "matrix_bytes_cycled": 4 * cells * len(mats)},
        "gvotes_per_s": round(total_votes / elapsed / 1e9, 3),
        "votes_per_event": round(float(np.mean(votes)), 1),
        "fill_gvotes_per_s": round(np.mean(votes) / fill_avg_s / 1e9, 3),
        "fill_kernel_ms": round(fill_avg_s * 1e3, 4),
        "stage_ms_events_every_stage": stage,
        "ms_per_step_without_events": round(1000.0 * (t3 - t2) / n_extra, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(tuning_now),
                     "kernel": "k_fill", "alg_bytes_per_launch": alg_bytes,
                     "fill_kernel_us": round(fill_avg_s * 1e6, 2),
                     "matrices_cycled": len(mats)},
        "single_matrix_loop": {
            "note": "one 256 MiB matrix rewritten every step: it stays in the 256 MB last-level "
                    "cache, so this is not an HBM figure",
            "events_per_s": round(args.steps / elapsed1, 2),
            "ms_per_step": round(1000.0 * elapsed1 / args.steps, 4),
            "fill_kernel_us": round(fill_avg1_s * 1e6, 2),
            "fill_alg_GBs": round(achieved1, 1),
            "frac_of_8TBs": round(achieved1 / HBM_PEAK_GBS, 4)},
        "peaks_per_event": round(float(np.mean(nfound)), 1),
        "tuning": tuning_now,
        "autotune": tuned,
    }
    # the plain baseline: zero the matrix, one global atomicAdd per vote (paper-style kernel)
    torch.cuda.synchronize()
    B.ht_profile_read("fill_atomic", reset=True)
    B.ht_profile_enable(True)
    for k in range(min(args.steps, 50)):
        x, y, z = dev_hits[k % args.events]
        B.ht_fill(spec, x, y, z, mats[k % len(mats)], stream, atomic=True)
    torch.cuda.synchronize()
    B.ht_profile_enable(False)
    fa_ms, fa_n = B.ht_profile_read("fill_atomic", reset=True)
    fa_s = fa_ms / 1e3 / max(fa_n, 1)
    line["plain_atomic_fill"] = {"ms": round(fa_s * 1e3, 4),
                                 "gvotes_per_s": round(np.mean(votes) / fa_s / 1e9, 3)}
    # plain per-event latency (launch to result on the host), one event at a time, hits resident
    lat = []
    for k in range(100):
        i = k % args.events
        x, y, z = dev_hits[i]
        ts = time.perf_counter()
        B.ht_fill_peaks(spec, x, y, z, mats[k % len(mats)], h_out[i], cap, h_nf[i:i + 1], stream)
        stream.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
    line["plain_latency_ms"] = {"p50": round(percentile(lat, 50), 4), "p99": round(percentile(lat, 99), 4)}
    # plain per-event path with the hit upload: hits in pinned host memory, copied to the device
    # (three arrays), fill and peaks, the peak list written to pinned host memory, synchronised;
    # one event at a time (the PCIe-inclusive rate)
    h_hits = [tuple(torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (e.x, e.y, e.z))
              for e in evs]
    lat = []
    t0 = time.perf_counter()
    for k in range(200):
        i = k % args.events
        x, y, z = dev_hits[i]
        ts = time.perf_counter()
        for d, h in zip((x, y, z), h_hits[i]):
            d.copy_(h, non_blocking=True)
        B.ht_fill_peaks(spec, x, y, z, mats[k % len(mats)], h_out[i], cap, h_nf[i:i + 1], stream)
        stream.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
    dt = time.perf_counter() - t0
    line["plain_with_upload"] = {"events_per_s": round(200 / dt, 1),
                                 "p50_ms": round(percentile(lat, 50), 4),
                                 "p99_ms": round(percentile(lat, 99), 4)}
    pk = measure_peaks(B, torch, 4 * cells)
    line["measured_peaks"] = pk
    line["fill_frac_of_measured_write"] = round(achieved / pk["hbm_write_GBs"], 4)
    line["single_matrix_loop"]["fill_frac_of_matrix_sized_write"] = round(
        achieved1 / pk["matrix_sized_buffer"]["write_GBs"], 4)
    line["fill_votes_vs_atomic_roofline"] = round(
        line["fill_gvotes_per_s"] / pk["atomic_rand_Gops"], 3)
    # physics check of the peak lists against the generator's truth (Fig. 1 analogue)
    from paper_1507_03074_amd import physics
    phys = []
    for i in range(min(args.events, 8)):
        x, y, z = dev_hits[i]
        B.ht_fill_peaks(spec, x, y, z, acc, out[i], cap, nf[i:i + 1], stream)
        tr = B.tracks_to_host(B.ht_readout(spec, out[i], nf[i:i + 1], cap), nf[i:i + 1], cap)
        phys.append(physics.evaluate(spec, tr, evs[i]))
    line["physics"] = {
        "events": len(phys),
        "efficiency": round(sum(p["found"] for p in phys) / max(1, sum(p["in_acceptance"] for p in phys)), 4),
        "fake_rate": round(sum(p["unmatched_peaks"] for p in phys) / max(1, sum(p["peaks"] for p in phys)), 4),
        "rho_resolution_ht": round(float(np.mean([p["rho_resolution_ht"] for p in phys])), 5),
        "phi_resolution_ht_mrad": round(1e3 * float(np.mean([p["phi_resolution_ht"] for p in phys])), 3),
        "rho_resolution_lsq_fit": round(float(np.mean([p["rho_resolution_fit"] for p in phys])), 6),
        "phi_resolution_lsq_fit_mrad": round(1e3 * float(np.mean([p["phi_resolution_fit"] for p in phys])), 4),
        "tracks_in_acceptance_per_event": round(float(np.mean([p["in_acceptance"] for p in phys])), 1)}
    log("sector variant")
    line["sectors"] = bench_sectors(B, torch, synth, evs, dev_hits, min(args.steps, 300))
    if not args.quick:
        line["two_streams"] = bench_two_streams(B, torch, spec, dev_hits, h_out, h_nf, cap, args.steps)
        del acc, out, mats
        torch.cuda.empty_cache()
        log("batched workload 2")
        line["batched"] = bench_batched(B, torch, synth, 2, 100, 20, 1 << 13, tune_batch=True)
        log("stress workload 4")
        line["stress"] = bench_batched(B, torch, synth, 4, 16, 5, 1 << 21, tune_batch=True)
        log("transfer study")
        line["transfers"] = bench_transfers(B, torch, synth, spec)
        log("served workload 3")
        line["served"] = bench_served(B, torch, synth, n_pool=128, n_warm=200, n_meas=2000,
                                      rates=(0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2), budget_gib=24,
                                      max_batch=8, n_streams=2)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb, _ = cpu_baseline(spec, workload, args.cpu_seconds)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
