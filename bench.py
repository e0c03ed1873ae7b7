#!/usr/bin/env python3
"""Benchmark: synapses built + calibrated per second on one MI355X.

A step is one pass of the whole hot path over the microcircuit-shaped
network (77,169 nodes in 8 populations, 64 fixed_total_number Connect calls,
3.0e8 synapses): reset the context, set the step's seed (steps cycle through
seeds 1..10, as the paper's timings average ten seeds), create the nodes,
issue every Connect call (generation kernels), then calibrate (radix-sort
passes and the group index).  Inputs are the call descriptions; nothing is
copied from the host inside the timed region.

Prints one JSON line (rank 0) with the throughput, mean (std) of the step
time over the seeds, the roofline of the dominant kernel measured with HIP
events on the context's stream (in the timed steps, events around that kernel
only; every kernel's time from as many builds again with events around each
launch), the same build for the two-population
network and the 4,096-call batch (plain, batched and graph forms), and the
CPU oracle timed on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "synapses built+calibrated/sec at 3e8 synapses; p50/p99 ng_connect latency"
HBM_PEAK_GBS = 8000.0
# paper, Table 2: A100 node connection 0.08 s + calibration 0.408 s for ~3e8 synapses
PAPER_A100_SYN_PER_S = 3.0e8 / (0.08 + 0.408)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Bytes the method must move per synapse (the path's 42: the 14-byte record
# written once by generation, read once and written once sorted by the
# calibration).  The calibration's 28 bytes are split evenly over the kernels
# that move every record (the scatter and LDS-sort passes of the sort); the
# counting, planning and index kernels get none.
SORT_PASS_KERNELS = ("msd_scatter_a", "msd_scatter_b", "msd_tiles_c", "downsweep")
GEN_KERNELS = ("generate", "generate_batch")


def algorithmic_bytes(kernel: str, n_syn: int, kernels: dict, steps: int = 1) -> float | None:
    """Algorithmic bytes of `kernel` per step, given the timed launches
    (name -> (launches, ms[, records])) so that the sort's share is split
    over its record-moving launches and generation's over the launches that
    made the synapses (records = synapses generated, over `steps` steps)."""
    if kernel in GEN_KERNELS:
        rec = kernels.get(kernel, ())
        return 14.0 * (rec[2] / steps if len(rec) > 2 and rec[2] else n_syn)
    if kernel in SORT_PASS_KERNELS:
        launches = sum(kernels[k][0] for k in SORT_PASS_KERNELS if k in kernels)
        return 28.0 * n_syn * kernels[kernel][0] / launches
    return None


def moved_bytes(kernel: str, n_syn: int, plan: dict) -> float | None:
    """Bytes the implementation's kernel reads and writes per step (records
    of 14 bytes in blocks, 8 bytes packed, 12 bytes unpacked between
    passes); a diagnostic next to the algorithmic figure."""
    if not plan or plan.get("msd", 0) != 2:
        return None
    a = 8.0 if plan["narrow_a"] else 12.0
    b = 8.0 if plan["narrow_b"] else 12.0
    per = {"msd_count_a": 4.0, "msd_scatter_a": 14.0 + a, "msd_count_b": 4.0,
           "msd_scatter_b": a + b, "msd_tiles_c": (b if plan["b2"] else a) + 14.0}.get(kernel)
    return None if per is None else per * n_syn


def kernels_fingerprint(kernel: str) -> str:
    """Hash of the source that holds `kernel` (the most-significant-digit
    sort file for its kernels, else the radix-sort section of the kernel
    file): traffic counters taken on one version do not describe another."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2306_09855_amd", "csrc")
    if kernel.startswith("msd_"):
        with open(os.path.join(csrc, "ng_msd.hip"), "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:16]
    with open(os.path.join(csrc, "ng_kernels.hip"), "rb") as f:
        src = f.read()
    a = src.find(b"// Radix sort: reduce-then-scan")
    b = src.find(b"// Device-wide exclusive scan")
    if a < 0 or b < a:
        raise RuntimeError("radix-sort section markers not found in ng_kernels.hip")
    return hashlib.sha256(src[a:b]).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if there is none or the kernels changed since it was taken."""
    import glob
    fp = kernels_fingerprint(kernel)
    for path in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.md")):
        for line in open(path):
            line = line.strip()
            if not line.startswith("{"):
                continue
            try:
                rec = json.loads(line)
            except ValueError:
                continue
            if rec.get("kernel") == kernel and rec.get("workload") == workload and rec.get("kernels_sha") == fp:
                return rec["bytes_per_launch"]
    return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(sample_syn: int, one_thread_syn: int) -> dict:
    """The oracle as it stands, timed on this host: the microcircuit call list
    scaled to sample_syn synapses on all cores the process may use (its
    threaded mode, byte-identical to the single-thread mode), and on one core
    for one_thread_syn synapses.  Generation of every call plus calibration."""
    import oracle
    from paper_2306_09855_amd import workloads as W

    def run(total, threads):
        wl = W.microcircuit(total=total)
        with oracle.threads(threads):
            t0 = time.perf_counter()
            oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
            dt = time.perf_counter() - t0
        return wl.n_syn, dt

    cores = max(1, len(os.sched_getaffinity(0)))
    log(f"cpu baseline: oracle on {sample_syn:.3g} synapses, {cores} threads ...")
    n_all, t_all = run(sample_syn, cores)
    log(f"cpu baseline: oracle on {one_thread_syn:.3g} synapses, 1 thread ...")
    n_one, t_one = run(one_thread_syn, 1)
    return {"value": n_all / t_all, "unit": "synapses/s", "cores": cores, "kind": "oracle",
            "seconds": round(t_all, 3), "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": (f"microcircuit populations (77,169 nodes), 64 fixed_total_number calls scaled to "
                       f"{n_all} synapses; generation + calibration, {cores} threads"),
            "single_thread": {"value": n_one / t_one, "seconds": round(t_one, 3), "synapses": n_one}}


def _events(trace):
    """(time, episode, kind, call, marshalled call arguments), by arrival time."""
    from paper_2306_09855_amd import ng
    ev = []
    for ei, ep in enumerate(trace):
        ev.append((ep.times[0], ei, "create", None, None))
        for j, c in enumerate(ep.calls):
            ev.append((ep.times[1 + j], ei, "connect", c, ng.call_args(c)))
        ev.append((ep.times[-2], ei, "calibrate", None, None))
        ev.append((ep.times[-1], ei, "close", None, None))
    ev.sort(key=lambda e: (e[0], e[1]))
    return ev


def _wait_until(t):
    while True:
        d = t - time.perf_counter()
        if d <= 0:
            return
        if d > 3e-4:
            time.sleep(d - 2e-4)


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def serve_run(trace, n_streams, arena_bytes, block_size):
    """The trace through the server: requests submitted at their arrival times."""
    import torch
    from paper_2306_09855_amd import ng
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    arena = ng.arena_for(arena_bytes)
    srv = ng.ng_server_create(ng.ng_server_config(block_size, 0.1, 0, 0, 0), arena, arena_bytes,
                              [s.cuda_stream for s in streams])
    sessions, tickets = {}, []
    events = _events(trace)
    t0 = time.perf_counter()
    for (t, ei, kind, c, args) in events:
        _wait_until(t0 + t)
        if kind == "create":
            sessions[ei] = ng.ng_session_open(srv, trace[ei].seed)
            tickets.append((ng.ng_submit_create_nodes(sessions[ei], trace[ei].n_nodes)[1], kind, 0))
        elif kind == "connect":
            tickets.append((ng.ng_submit_connect(sessions[ei], *args), kind, c.n_syn()))
        elif kind == "calibrate":
            tickets.append((ng.ng_submit_calibrate(sessions[ei]), kind, 0))
        else:
            tickets.append((ng.ng_submit_close(sessions[ei]), kind, 0))
    submit_s = time.perf_counter() - t0
    lat, first, last, syn, bad = [], None, 0, 0, 0
    for (tk, kind, n) in tickets:
        info = ng.ng_wait(srv, tk)
        bad += info.status != 0
        first = info.arrival_ns if first is None else min(first, info.arrival_ns)
        last = max(last, info.done_ns)
        if kind == "connect":
            lat.append((info.done_ns - info.arrival_ns) / 1e6)
            syn += n
    stats = ng.ng_server_get_stats(srv)
    ng.ng_server_destroy(srv)
    del arena
    torch.cuda.empty_cache()
    span = (last - first) / 1e9
    return {"synapses": syn, "seconds": round(span, 4), "synapses_per_s": syn / span,
            "connect_p50_ms": _pct(lat, 50), "connect_p99_ms": _pct(lat, 99), "failed": bad,
            "launches": stats["launches"], "calls_per_launch": round(stats["packed_calls"] / max(stats["launches"], 1), 2),
            "calibrate_packs": stats["calibrate_packs"], "max_sessions_per_pack": stats["max_sessions_per_pack"],
            "client_submit_s": round(submit_s, 4), "scheduler_busy_s": round(stats["scheduler_busy_ns"] / 1e9, 4),
            "scheduler_launch_s": round(stats["host_launch_ns"] / 1e9, 4),
            "scheduler_calibrate_s": round(stats["host_calibrate_ns"] / 1e9, 4),
            "peak_arena_GiB": round(stats["peak_arena_bytes"] / 2**30, 2)}


def plain_run(trace, block_size, pool):
    """The same trace served one request at a time, each synchronized (FIFO).
    pool: arena tensors by size, reused across episodes and runs."""
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import arena_bytes_for
    stream = torch.cuda.Stream()
    ctxs, arenas, lat, syn = {}, {}, [], 0
    events = _events(trace)
    t0 = time.perf_counter()
    first = last = None
    for (t, ei, kind, c, args) in events:
        arrival = t0 + t
        _wait_until(arrival)
        ep = trace[ei]
        if kind == "create":
            need = arena_bytes_for(ep.n_syn, ep.n_nodes, 63, block_size, 9)
            size = 1 << max(24, (need - 1).bit_length())
            free = pool.setdefault(size, [])
            a = free.pop() if free else ng.arena_for(size)
            arenas[ei] = a
            ctxs[ei] = ng.ng_create(ng.ng_config(block_size, ep.seed, 0.1, 0), a, size, stream.cuda_stream)
            ng.ng_create_nodes(ctxs[ei], ep.n_nodes)
        elif kind == "connect":
            ng.ng_connect(ctxs[ei], *args)
            ng.ng_sync(ctxs[ei])
            syn += c.n_syn()
        elif kind == "calibrate":
            ng.ng_calibrate(ctxs[ei])
            ng.ng_sync(ctxs[ei])
        else:
            ng.ng_destroy(ctxs.pop(ei))
            a = arenas.pop(ei)
            pool[a.numel()].append(a)
        done = time.perf_counter()
        first = arrival if first is None else min(first, arrival)
        last = done
        if kind == "connect":
            lat.append((done - arrival) * 1e3)
    for ei, c in ctxs.items():
        ng.ng_destroy(c)
        a = arenas.pop(ei)
        pool[a.numel()].append(a)
    span = last - first
    return {"synapses": syn, "seconds": round(span, 4), "synapses_per_s": syn / span,
            "connect_p50_ms": _pct(lat, 50), "connect_p99_ms": _pct(lat, 99)}


def serving_bench(n_streams=4, block_size=1 << 20, loads=(0.5, 1.0, 2.0, 4.0), burst_episodes=2,
                  sweep_episodes=15, arena_bytes=128 << 30):
    """Serving form against the plain sequential path.

    capacity: a backlog (every request of 32 clients x burst_episodes sessions
    at time 0): synapses/s of both paths.
    sweep: Poisson arrivals (32 clients x sweep_episodes sessions, about 10,000
    requests) at each load x the plain path's request capacity: p50/p99
    Connect latency (arrival to device completion) and synapses/s of both."""
    import torch
    from paper_2306_09855_amd import workloads as W
    pool = {}
    warm = W.serving_trace(n_slots=8, episodes_per_slot=1, burst=True, gen_seed=6)
    serve_run(warm, n_streams, arena_bytes, block_size)
    burst = W.serving_trace(episodes_per_slot=burst_episodes, burst=True)
    n_req = sum(len(e.calls) + 3 for e in burst)
    total = sum(e.n_syn for e in burst)
    log(f"serving: backlog of {len(burst)} sessions, {n_req} requests, {total:.3g} synapses")
    plain_cap = plain_run(burst, block_size, pool)
    served_cap = serve_run(burst, n_streams, arena_bytes, block_size)
    log(f"serving: backlog plain {plain_cap['seconds']} s, served {served_cap['seconds']} s")
    plain_rate = n_req / plain_cap["seconds"]
    # the plain path holds one arena per open session: allocate them untimed,
    # at the highest load (the most sessions open at once)
    plain_run(W.serving_trace(episodes_per_slot=sweep_episodes, rate=max(loads) * plain_rate), block_size, pool)
    sweep = []
    for load in loads:
        timed = W.serving_trace(episodes_per_slot=sweep_episodes, rate=load * plain_rate)
        n_t = sum(len(e.calls) + 3 for e in timed)
        p = plain_run(timed, block_size, pool)
        sv = serve_run(timed, n_streams, arena_bytes, block_size)
        sweep.append({"load_vs_plain_capacity": load, "rate_req_per_s": round(load * plain_rate, 1),
                      "requests": n_t, "plain": p, "served": sv})
        log(f"serving: load {load}: {n_t} requests, connect p50/p99 plain {p['connect_p50_ms']:.3g}/"
            f"{p['connect_p99_ms']:.3g} ms, served {sv['connect_p50_ms']:.3g}/{sv['connect_p99_ms']:.3g} ms")
    pool.clear()
    torch.cuda.empty_cache()
    return {"clients": 32, "streams": n_streams, "block_size": block_size, "arena_GiB": arena_bytes / 2**30,
            "backlog": {"sessions": len(burst), "requests": n_req, "synapses": total,
                        "served": served_cap, "plain": plain_cap,
                        "speedup": round(served_cap["synapses_per_s"] / plain_cap["synapses_per_s"], 2)},
            "sweep": sweep}


def copass_bench(wl, block_size: int, steps: int, warmup: int, radix_bits: int, sort_ranges: int) -> dict:
    """The same build with the COPASS in-place block sort as calibration:
    time per step, per-kernel times, the copies' bandwidth and peak arena use."""
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    arena = arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, block_size, 9)
    side = torch.cuda.Stream()
    net = Network(wl.seed, wl.h, block_size, arena, stream=side.cuda_stream)
    net.tune(radix_bits, sort_ranges)
    net.set_calibration("copass")
    ctx = net.ctx
    calls = [ng.call_args(c) for c in wl.calls]

    def step():
        ng.ng_reset(ctx)
        for n in wl.populations:
            ng.ng_create_nodes(ctx, n)
        for a in calls:
            ng.ng_connect(ctx, *a)
        ng.ng_calibrate(ctx)

    for _ in range(warmup):
        step()
    ng.ng_sync(ctx)
    ng.ng_enable_timing(ctx, True)
    ng.ng_read_timing(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    ng.ng_sync(ctx)
    t1 = time.perf_counter()
    kernels = ng.ng_read_timing(ctx, reset=True, records=True)
    ng.ng_enable_timing(ctx, False)
    peak = net.memory_stats()[1]
    net.close()
    ms = 1e3 * (t1 - t0) / steps
    per = {}
    for name, (launches, total_ms, recs) in kernels.items():
        k_ms = total_ms / steps
        gbps = None
        if name == "copass_copy" and k_ms > 0:
            gbps = round(26.0 * recs / steps / (k_ms / 1e3) / 1e9, 1)  # read 14 + write 12 bytes, or 12 + 14
        per[name] = {"launches_per_step": launches / steps, "ms_per_step": round(k_ms, 4), "GBps_algorithmic": gbps}
        if name == "copass_copy":
            per[name]["records_per_step"] = recs / steps
    gen_ms = sum(per.get(k, {}).get("ms_per_step", 0.0) for k in GEN_KERNELS)
    return {"ms_per_step": round(ms, 3), "synapses_per_s": wl.n_syn / (ms / 1e3),
            "calibrate_device_ms": round(sum(v["ms_per_step"] for v in per.values()) - gen_ms, 3),
            "block_size": block_size, "blocks": -(-wl.n_syn // block_size),
            "peak_arena_GiB": round(peak / 2**30, 3), "kernels": per}


def arrays_bench(wl, block_size: int, steps: int, warmup: int, radix_bits: int, sort_ranges: int) -> dict:
    """The same build with every call's source group given as an index array
    (a random permutation of its population) and per-connection weights and
    delays (ng_connect_groups): time per step and the bandwidth of the
    generation that maps each synapse through the arrays."""
    import numpy as np
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    arena = arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, block_size, 9)
    side = torch.cuda.Stream()
    net = Network(wl.seed, wl.h, block_size, arena, stream=side.cuda_stream)
    net.tune(radix_bits, sort_ranges)
    ctx = net.ctx
    g = torch.Generator(device="cuda").manual_seed(1)
    args = []
    for c in wl.calls:
        s0, ns = c.src
        idx = (torch.randperm(ns, device="cuda", generator=g) + s0).to(torch.int32)
        n = c.n_syn()
        w = torch.randn(n, device="cuda", generator=g) * 0.05 + 0.5
        d = torch.rand(n, device="cuda", generator=g) * 3.0  # ms: 1..30 steps at h = 0.1
        args.append((ng.group(idx), ng.group(c.tgt), ng.conn_spec(c.rule, c.k_or_n),
                     ng.syn_spec(c.weight, c.delay), w, d, idx))
    torch.cuda.synchronize()

    def step():
        ng.ng_reset(ctx)
        for n in wl.populations:
            ng.ng_create_nodes(ctx, n)
        for a in args:
            ng.ng_connect_groups(ctx, *a[:4], a[4], a[5])
        ng.ng_calibrate(ctx)

    for _ in range(warmup):
        step()
    ng.ng_sync(ctx)
    ng.ng_enable_timing(ctx, True)
    ng.ng_read_timing(ctx, reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    ng.ng_sync(ctx)
    t1 = time.perf_counter()
    kernels = ng.ng_read_timing(ctx, reset=True)
    ng.ng_enable_timing(ctx, False)
    net.close()
    ms = 1e3 * (t1 - t0) / steps
    # generation per connection: the 14-byte record written, the source index,
    # weight and delay (ms) read from the arrays
    ab = 26.0 * wl.n_syn
    per = {}
    for name, (launches, total_ms) in kernels.items():
        k_ms = total_ms / steps
        per[name] = {"launches_per_step": launches / steps, "ms_per_step": round(k_ms, 4),
                     "GBps_algorithmic": round(ab / (k_ms / 1e3) / 1e9, 1) if name == "generate" and k_ms else None}
    return {"ms_per_step": round(ms, 3), "synapses_per_s": wl.n_syn / (ms / 1e3),
            "arrays": "source index arrays (permuted populations), per-connection weights and delays",
            "generate_bytes_per_connection": 26, "kernels": per}


def no_autapse_bench(wl, block_size: int, steps: int, warmup: int, radix_bits: int, sort_ranges: int,
                     multapses: int = 1) -> dict:
    """The same build with allow_autapses = 0 on every call (the calls whose
    source and target populations are the same draw without self-pairs);
    with multapses = 0 also without repeated pairs (keyed permutations)."""
    import types
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    arena = arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, block_size, 9)
    side = torch.cuda.Stream()
    net = Network(wl.seed, wl.h, block_size, arena, stream=side.cuda_stream)
    net.tune(radix_bits, sort_ranges)
    ctx = net.ctx
    calls = [ng.call_args(types.SimpleNamespace(rule=c.rule, src=c.src, tgt=c.tgt, k_or_n=c.k_or_n,
                                                weight=c.weight, delay=c.delay, allow_autapses=0,
                                                allow_multapses=multapses))
             for c in wl.calls]
    overlapping = sum(1 for c in wl.calls if c.src[0] < c.tgt[0] + c.tgt[1] and c.tgt[0] < c.src[0] + c.src[1])

    def step():
        ng.ng_reset(ctx)
        for n in wl.populations:
            ng.ng_create_nodes(ctx, n)
        for a in calls:
            ng.ng_connect(ctx, *a)
        ng.ng_calibrate(ctx)

    for _ in range(warmup):
        step()
    ng.ng_sync(ctx)
    ng.ng_enable_timing(ctx, True)
    ng.ng_read_timing(ctx, reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    ng.ng_sync(ctx)
    t1 = time.perf_counter()
    kernels = ng.ng_read_timing(ctx, reset=True)
    ng.ng_enable_timing(ctx, False)
    n_conns = ng.ng_get_connections(ctx).n_conns
    net.close()
    ms = 1e3 * (t1 - t0) / steps
    gen_ms = sum(kernels.get(k, (0, 0.0))[1] for k in GEN_KERNELS)
    return {"ms_per_step": round(ms, 3), "synapses": n_conns, "synapses_per_s": n_conns / (ms / 1e3),
            "calls_with_overlapping_ranges": overlapping,
            "generate_ms_per_step": round(gen_ms / steps, 4)}


def pairwise_bench(wl, block_size: int, steps: int, warmup: int, radix_bits: int, sort_ranges: int,
                   n_tgt: int = 50_000, p: float = 0.0777) -> dict:
    """One pairwise_bernoulli call from all nodes of the workload to the
    first n_tgt of them (~3e8 connections), calibrated: counting pass,
    exact reservation, writing pass, sort and index."""
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    n_exp = int(wl.n_nodes * n_tgt * p)
    arena = arena_bytes_for(int(n_exp * 1.01), wl.n_nodes, wl.max_delay, block_size, 9) + (64 << 20)
    side = torch.cuda.Stream()
    net = Network(wl.seed, wl.h, block_size, arena, stream=side.cuda_stream)
    net.tune(radix_bits, sort_ranges)
    ctx = net.ctx
    conn = ng.conn_spec("pairwise_bernoulli", 0, p=p)
    syn = ng.syn_spec(("normal", 0.5, 0.05), ("uniform_int", 1, 30))
    n = 0

    def step():
        nonlocal n
        ng.ng_reset(ctx)
        ng.ng_create_nodes(ctx, wl.n_nodes)
        n = ng.ng_connect(ctx, ng.ng_range(0, wl.n_nodes), ng.ng_range(0, n_tgt), conn, syn)[2]
        ng.ng_calibrate(ctx)

    for _ in range(warmup):
        step()
    ng.ng_sync(ctx)
    ng.ng_enable_timing(ctx, True)
    ng.ng_read_timing(ctx, reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    ng.ng_sync(ctx)
    t1 = time.perf_counter()
    kernels = ng.ng_read_timing(ctx, reset=True)
    ng.ng_enable_timing(ctx, False)
    net.close()
    ms = 1e3 * (t1 - t0) / steps
    per = {k: round(v[1] / steps, 4) for k, v in kernels.items()}
    pairs = wl.n_nodes * n_tgt
    return {"pairs": pairs, "p": p, "connections": n, "ms_per_step": round(ms, 3),
            "synapses_per_s": n / (ms / 1e3), "pairs_per_s_counting": pairs / (per.get("pb_count", 0) / 1e3)
            if per.get("pb_count") else None, "kernels_ms_per_step": per}


def delivery_bench(wl, block_size: int, rate_per_step: float = 1e-3, warm_steps: int = 100,
                   steps: int = 500) -> dict:
    """Spike buffers and delivery over the calibrated network: random spike
    trains with `rate_per_step` spikes per node and step (10 Hz at 0.1 ms),
    `warm_steps` steps to fill the queues, then `steps` timed steps."""
    import numpy as np
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    arena = arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, block_size, 9) + (512 << 20)
    side = torch.cuda.Stream()
    net = Network(wl.seed, wl.h, block_size, arena, stream=side.cuda_stream)
    net.build(wl)
    net.spikes_init()
    gp, gs = net.group_index()
    outdeg = gs[gp[1:].astype(np.int64)].astype(np.int64) - gs[gp[:-1].astype(np.int64)].astype(np.int64)
    rng = np.random.default_rng(7)
    trains = [np.nonzero(rng.random(wl.n_nodes) < rate_per_step)[0] for _ in range(warm_steps + steps)]
    dev = [torch.from_numpy(t.astype(np.int32)).cuda() for t in trains]
    inp = torch.zeros(wl.n_nodes, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ctx = net.ctx
    for t in range(warm_steps):
        ng.ng_spikes_step(ctx, dev[t], None, dev[t].numel(), inp)
    ng.ng_sync(ctx)
    ng.ng_enable_timing(ctx, True)
    ng.ng_read_timing(ctx, reset=True)
    t0 = time.perf_counter()
    for t in range(warm_steps, warm_steps + steps):
        ng.ng_spikes_step(ctx, dev[t], None, dev[t].numel(), inp)
    ng.ng_sync(ctx)
    t1 = time.perf_counter()
    kernels = ng.ng_read_timing(ctx, reset=True)
    ng.ng_enable_timing(ctx, False)
    net.close()
    emitted = sum(int(outdeg[t].sum()) for t in trains[warm_steps:])
    wall = t1 - t0
    dev_ms = kernels.get("spikes_step", (steps, 0.0))[1]
    return {"steps": steps, "spikes_per_step": round(sum(len(t) for t in trains[warm_steps:]) / steps, 1),
            "us_per_step": round(1e6 * wall / steps, 2), "device_us_per_step": round(1e3 * dev_ms / steps, 2),
            "connections_delivered_per_s": emitted / wall,
            "delivered_note": "out-degree of the spikes emitted in the timed steps",
            "GBps_algorithmic": round(8.0 * emitted / (dev_ms / 1e3) / 1e9, 1) if dev_ms else None}


SEEDS = tuple(range(1, 11))  # the paper's timings are means over ten seeds


def form_bench(wl, form: str, steps: int, warmup: int, block_size: int) -> dict:
    """One workload built and calibrated in the plain form (one ng_connect
    per call; the context queues small calls and launches them together), the
    plain form with the queue off (plain_unqueued: one generation launch per
    call), the batched form (one ng_connect_batch) or the graph form (the
    batched build captured once, replayed with each step's seed); steps cycle
    through the seeds.  Wall time per step."""
    import torch
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    arena = arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, block_size, 9)
    side = torch.cuda.Stream()
    net = Network(wl.seed, wl.h, block_size, arena, stream=side.cuda_stream)
    ctx = net.ctx
    if form == "plain_unqueued":
        ng.ng_set_schedule(ctx, {**ng.ng_get_schedule(ctx), "queued_calls": 0})
    calls = [ng.call_args(c) for c in wl.calls]
    batch = [list(x) for x in zip(*calls)]

    def build():
        for n in wl.populations:
            ng.ng_create_nodes(ctx, n)
        if form in ("plain", "plain_unqueued"):
            for a in calls:
                ng.ng_connect(ctx, *a)
        else:
            ng.ng_connect_batch(ctx, *batch)
        ng.ng_calibrate(ctx)

    graph = None
    if form == "graph":
        ng.ng_reset(ctx)
        ng.ng_graph_begin(ctx)
        build()
        graph = ng.ng_graph_end(ctx)

    def step(i):
        seed = SEEDS[i % len(SEEDS)]
        if graph is not None:
            ng.ng_graph_launch(graph, seed)
        else:
            ng.ng_reset(ctx)
            ng.ng_set_seed(ctx, seed)
            build()

    for i in range(warmup):
        step(i)
    ng.ng_sync(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    ng.ng_sync(ctx)
    t1 = time.perf_counter()
    if graph is not None:
        ng.ng_graph_destroy(graph)
    net.close()
    torch.cuda.empty_cache()
    ms = 1e3 * (t1 - t0) / steps
    return {"form": form, "ms_per_step": round(ms, 3), "synapses_per_s": wl.n_syn / (ms / 1e3)}


def workload_legs(block_size: int, steps: int) -> dict:
    """The two-population network (four calls, four rules, 1.54e8 synapses)
    in the plain form, and the 4,096-call batch (~4.3e8 synapses, mixed rules
    over 1e6 nodes) in every form: vs_plain compares with the plain form (its
    calls queued and launched together), vs_one_launch_per_call with the plain
    form whose queue is off."""
    from paper_2306_09855_amd import workloads as W
    out = {}
    tp = W.two_pop_mixed()
    out["two_population"] = {"n_syn": tp.n_syn, "n_calls": len(tp.calls), "n_nodes": tp.n_nodes,
                             "plain": form_bench(tp, "plain", steps, 1, block_size)}
    log(f"two-population network: {out['two_population']['plain']['ms_per_step']} ms/step")
    bm = W.batch_mixed()
    legs = {f: form_bench(bm, f, steps, 1, block_size) for f in ("plain", "plain_unqueued", "batched", "graph")}
    for f in ("plain", "batched", "graph"):
        legs[f]["vs_one_launch_per_call"] = round(legs[f]["synapses_per_s"] / legs["plain_unqueued"]["synapses_per_s"], 2)
    for f in ("batched", "graph"):
        legs[f]["vs_plain"] = round(legs[f]["synapses_per_s"] / legs["plain"]["synapses_per_s"], 2)
    out["batch_4096"] = {"n_syn": bm.n_syn, "n_calls": len(bm.calls), "n_nodes": bm.n_nodes, **legs}
    log("batch of 4,096 calls: " + ", ".join(f"{f} {legs[f]['ms_per_step']} ms" for f in legs))
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps (seeds 1..10 in turn)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="microcircuit", choices=["microcircuit", "batch_mixed"],
                    help="microcircuit: 64 calls, 3.0e8 synapses; batch_mixed: 4,096 uneven calls, ~4.3e8")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "graph"],
                    help="plain: one ng_connect per call; batched: one ng_connect_batch; "
                         "graph: the batched build captured once and replayed")
    ap.add_argument("--calibration", default="radix", choices=["radix", "lsd", "msd"],
                    help="radix: the default form choice; lsd / msd: force one form")
    ap.add_argument("--tune", type=int, default=1,
                    help="pick the kernel schedule with the autotuner first (untimed); 0 keeps the default")
    ap.add_argument("--radix-bits", type=int, default=9, help="widest digit of the LSD form (fewest passes)")
    ap.add_argument("--sort-ranges", type=int, default=1024, help="static ranges (workgroups) of each scatter pass")
    ap.add_argument("--block-size", type=int, default=1 << 24)
    ap.add_argument("--cpu-sample", type=float, default=3.0e8,
                    help="synapses of the oracle run on all cores; 0 skips the CPU baseline")
    ap.add_argument("--cpu-one-thread", type=float, default=3.0e7, help="synapses of the single-thread oracle run")
    ap.add_argument("--total", type=float, default=3.0e8)
    ap.add_argument("--legs", type=int, default=1,
                    help="also time the two-population network and the 4,096-call batch in every form")
    ap.add_argument("--no-autapses", type=int, default=1,
                    help="also time the build with allow_autapses = 0 on every call")
    ap.add_argument("--pairwise", type=int, default=1,
                    help="also time a ~3e8-connection pairwise_bernoulli build")
    ap.add_argument("--delivery", type=int, default=1,
                    help="also time spike delivery (Sec. 2.3) over the calibrated network")
    ap.add_argument("--arrays", type=int, default=1,
                    help="also time the build with index arrays and per-connection weights/delays")
    ap.add_argument("--copass", type=int, default=1,
                    help="also time the COPASS in-place calibration on the same build (plain form)")
    ap.add_argument("--serve", type=int, default=1,
                    help="also run the serving trace (32 sessions; p50/p99 Connect latency); 0 skips")
    ap.add_argument("--copy-probe", type=float, default=0,
                    help="only run a plain device copy of this many bytes (calibrates counter readings)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; sharding over several GPUs is not implemented",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch
    if args.copy_probe:
        n = int(args.copy_probe)
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n}))
        return 0
    from paper_2306_09855_amd import ng
    from paper_2306_09855_amd import workloads as W
    from paper_2306_09855_amd.network import Network, arena_bytes_for

    torch.cuda.set_device(0)
    if args.workload == "microcircuit":
        wl = W.microcircuit(total=int(args.total))
    else:
        wl = W.batch_mixed()
    n_syn = wl.n_syn
    arena = arena_bytes_for(n_syn, wl.n_nodes, wl.max_delay, args.block_size, 9)
    log(f"workload {wl.name}: {wl.n_nodes} nodes, {len(wl.calls)} calls, {n_syn:.3g} synapses, "
        f"arena {arena / 2**30:.1f} GiB, form {args.form}")
    side = torch.cuda.Stream()  # graphs cannot capture the null stream
    net = Network(wl.seed, wl.h, args.block_size, arena, stream=side.cuda_stream)
    ctx = net.ctx
    schedule = {"calibration": args.calibration, "radix_bits": args.radix_bits, "sort_ranges": args.sort_ranges,
                "msd_tile": 16384, "gen_synapses_per_lane": 4, "queued_calls": 256}
    schedule_source = "default"
    if args.tune and args.calibration == "radix":
        from paper_2306_09855_amd.autotune import tune
        t0 = time.perf_counter()
        schedule, cached = tune(net, wl, batched=args.form != "plain", use_cache=False)
        schedule_source = f"autotuner ({time.perf_counter() - t0:.1f} s, untimed)"
        log(f"autotuner: {schedule}")
    ng.ng_set_schedule(ctx, schedule)
    calls = [ng.call_args(c) for c in wl.calls]
    batch = [list(x) for x in zip(*calls)]

    def build():
        for n in wl.populations:
            ng.ng_create_nodes(ctx, n)
        if args.form == "plain":
            for a in calls:
                ng.ng_connect(ctx, *a)
        else:
            ng.ng_connect_batch(ctx, *batch)
        ng.ng_calibrate(ctx)

    graph = None
    if args.form == "graph":
        ng.ng_reset(ctx)
        ng.ng_graph_begin(ctx)
        build()
        graph = ng.ng_graph_end(ctx)

    def step(i):
        seed = SEEDS[i % len(SEEDS)]
        if graph is not None:
            ng.ng_graph_launch(graph, seed)
        else:
            ng.ng_reset(ctx)
            ng.ng_set_seed(ctx, seed)
            build()

    for i in range(args.warmup):
        step(i)
        ng.ng_sync(ctx)
        log(f"warmup {i + 1}/{args.warmup} done")

    def kernel_times():
        """Per-kernel times: as many eager builds again, untimed, with an
        event pair around every launch (each pair leaves the GPU idle for a
        few microseconds); the longest kernel in all is the dominant one."""
        ng.ng_time_only(ctx, None)
        ng.ng_enable_timing(ctx, True)
        ng.ng_read_timing(ctx, reset=True)
        for i in range(args.steps):
            ng.ng_reset(ctx)
            ng.ng_set_seed(ctx, SEEDS[i % len(SEEDS)])
            build()
        k = ng.ng_read_timing(ctx, reset=True, records=True)
        ng.ng_enable_timing(ctx, False)
        return k, (max(k.items(), key=lambda kv: kv[1][1])[0] if k else None)

    # The timed steps carry events around the dominant kernel only.  Graph
    # replays carry none: the graph form's kernel times are those of eager
    # builds after the replays (the context is frozen while its graph lives).
    kernels, dom, dom_timed = {}, None, None
    if graph is None:
        kernels, dom = kernel_times()
        if dom is not None:
            ng.ng_time_only(ctx, dom)
            ng.ng_enable_timing(ctx, True)
            ng.ng_read_timing(ctx, reset=True)
    stream = torch.cuda.ExternalStream(net.stream) if net.stream else torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step(i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if dom is not None:
        dom_timed = ng.ng_read_timing(ctx, reset=True, records=True).get(dom)
        ng.ng_enable_timing(ctx, False)
        ng.ng_time_only(ctx, None)
    if graph is not None:
        ng.ng_graph_destroy(graph)
        graph = None
        kernels, dom = kernel_times()
    log(f"timed {args.steps} steps in {t1 - t0:.4f} s")

    wall = t1 - t0
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    dev_ms = float(step_ms.sum())
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps * n_syn / wall

    plan = ng.ng_calibration_plan(n_syn, wl.n_nodes, wl.max_delay, schedule["sort_ranges"])
    cal = schedule["calibration"]
    msd = plan["msd"] == 2 and cal == "radix" or (cal == "msd" and plan["msd"] >= 1)
    dbits = int(wl.max_delay).bit_length()
    sbits = int(wl.n_nodes - 1).bit_length()
    lsd_passes = max(1, -(-(sbits + dbits) // schedule["radix_bits"]))
    per_kernel = {}
    for name, (launches, total_ms, _) in kernels.items():
        ms = total_ms / args.steps
        ab = algorithmic_bytes(name, n_syn, kernels, args.steps)
        mb = moved_bytes(name, n_syn, plan) if msd else None
        per_kernel[name] = {"launches_per_step": launches / args.steps, "ms_per_step": round(ms, 4),
                            "GBps_algorithmic": None if ab is None or ms == 0 else round(ab / ms / 1e6, 1),
                            "GBps_moved": None if mb is None or ms == 0 else round(mb / ms / 1e6, 1)}
    roofline = None
    if dom is not None:
        launches, total_ms = (dom_timed or kernels[dom])[:2]
        ab_step = algorithmic_bytes(dom, n_syn, kernels, args.steps)
        if ab_step is not None:
            per_launch_bytes = ab_step * args.steps / launches
            avg_s = total_ms / launches / 1e3
            achieved = per_launch_bytes / avg_s / 1e9
            mb = moved_bytes(dom, n_syn, plan) if msd else None
            roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(dom, wl.name),
                        "bytes_per_launch": per_launch_bytes, "avg_launch_ms": round(avg_s * 1e3, 4),
                        "avg_launch_from": "HIP events around the kernel's launches in the timed steps"
                        if dom_timed else "HIP events around every launch of eager builds after the graph replays",
                        "bytes_note": "the method's 28 bytes per synapse of calibration split evenly over the "
                                      "sort's record-moving launches (14 per synapse for generation)",
                        "moved_bytes_per_launch": None if mb is None else mb * args.steps / launches}
    path_alg = 42.0 * n_syn  # write each record once, read it and write it sorted once
    if msd:
        calib = {"form": "msd", "digits": [plan["b1"], plan["b2"], plan["b3"]],
                 "packed_after_a": plan["narrow_a"], "packed_after_b": plan["narrow_b"]}
    else:
        calib = {"form": "lsd", "radix_bits": schedule["radix_bits"], "passes": lsd_passes}
    result = {
        "metric": METRIC, "value": value, "unit": "synapses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / PAPER_A100_SYN_PER_S, 2) if wl.name == "microcircuit" and n_syn == 3e8 else None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": wl.name, "n_nodes": wl.n_nodes, "n_calls": len(wl.calls),
                   "n_syn": n_syn,
                   "rule": "fixed_total_number" if wl.name == "microcircuit" else "mixed",
                   "delays": f"uniform_int 1..{wl.max_delay}",
                   "weights": "normal fp32", "form": args.form, "seeds": list(SEEDS),
                   "block_size": args.block_size, "calibration": calib,
                   "schedule": schedule, "schedule_source": schedule_source},
        "device_ms_per_step": round(dev_ms / args.steps, 4),
        "step_ms_over_seeds": {"mean": round(float(step_ms.mean()), 4), "std": round(float(step_ms.std(ddof=1)), 4)
                               if args.steps > 1 else 0.0, "steps": args.steps,
                               "note": "device time of each step (HIP events), steps cycling through the seeds"},
        "path_roofline": {"algorithmic_bytes_per_step": path_alg,
                          "frac": round(path_alg / (ms_per_step / 1e3) / (HBM_PEAK_GBS * 1e9), 4)},
        "roofline": roofline,
        "kernels": per_kernel,
        "kernels_note": "per-kernel times from as many eager builds again, untimed (before the timed steps; after "
                        "the replays for the graph form), with HIP events around every launch; the timed steps "
                        "carry events around the dominant kernel only",
    }
    radix_peak = net.memory_stats()[1]
    net.close()
    del net
    torch.cuda.empty_cache()
    legs_steps = max(1, min(args.steps, 3))
    if args.legs and args.form == "plain" and wl.name == "microcircuit":
        # the same build with ng_connect's queue off: one generation launch per call
        one = form_bench(wl, "plain_unqueued", legs_steps, 1, args.block_size)
        result["one_launch_per_call"] = {**one, "note": "the headline build with queued_calls = 0"}
        log(f"one launch per call: {one['ms_per_step']} ms/step")
        result.update(workload_legs(args.block_size, legs_steps))
    if args.copass and args.form == "plain":
        cp = copass_bench(wl, args.block_size, legs_steps, 1, args.radix_bits, args.sort_ranges)
        cp["radix_peak_arena_GiB"] = round(radix_peak / 2**30, 3)
        log(f"copass: {cp['ms_per_step']} ms/step, peak arena {cp['peak_arena_GiB']} GiB "
            f"(radix {cp['radix_peak_arena_GiB']} GiB)")
        result["copass"] = cp
        torch.cuda.empty_cache()
    if args.arrays and args.form == "plain" and wl.name == "microcircuit":
        ar = arrays_bench(wl, args.block_size, legs_steps, 1, args.radix_bits, args.sort_ranges)
        log(f"arrays: {ar['ms_per_step']} ms/step")
        result["arrays"] = ar
        torch.cuda.empty_cache()
    if args.no_autapses and args.form == "plain" and wl.name == "microcircuit":
        na = no_autapse_bench(wl, args.block_size, legs_steps, 1, args.radix_bits, args.sort_ranges)
        log(f"no autapses: {na['ms_per_step']} ms/step, generate {na['generate_ms_per_step']} ms")
        result["no_autapses"] = na
        nm = no_autapse_bench(wl, args.block_size, legs_steps, 1, args.radix_bits, args.sort_ranges,
                              multapses=0)
        log(f"no autapses, no multapses: {nm['ms_per_step']} ms/step, generate {nm['generate_ms_per_step']} ms")
        result["no_autapses_no_multapses"] = nm
        torch.cuda.empty_cache()
    if args.pairwise and args.form == "plain" and wl.name == "microcircuit":
        pb = pairwise_bench(wl, args.block_size, legs_steps, 1, args.radix_bits, args.sort_ranges)
        log(f"pairwise_bernoulli: {pb['ms_per_step']} ms/step, {pb['connections']} connections")
        result["pairwise_bernoulli"] = pb
        torch.cuda.empty_cache()
    if args.delivery and args.form == "plain" and wl.name == "microcircuit":
        dl = delivery_bench(wl, args.block_size)
        log(f"delivery: {dl['us_per_step']} us/step, {dl['connections_delivered_per_s']:.3g} connections/s")
        result["delivery"] = dl
        torch.cuda.empty_cache()
    if args.serve:
        sv = serving_bench()
        result["serving"] = sv
        at1 = next(x for x in sv["sweep"] if x["load_vs_plain_capacity"] == 1.0)
        result["latency_p50_ms"] = at1["served"]["connect_p50_ms"]
        result["latency_p99_ms"] = at1["served"]["connect_p99_ms"]
        result["latency_load"] = "Poisson arrivals at the plain path's capacity, served form"
    if args.cpu_sample > 0 and wl.name == "microcircuit":
        result["cpu_baseline"] = cpu_baseline(int(args.cpu_sample), int(args.cpu_one_thread))
    print(json.dumps(result))
    return 0


if __name__ == "__main__":
    sys.exit(main())
