"""Autotuner for the calibration schedule (radix digit width, range count).

For a workload it times the calibration kernels under a few schedules, keeps
the fastest and caches the choice as JSON per device, keyed by the connection
count (rounded to a power of two) and the key width.  Results never depend on
the schedule, only the speed does.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import ng

CANDIDATES = [(7, 1024), (8, 512), (8, 1024), (8, 2048), (9, 1024), (9, 2048)]
SORT_KERNELS = ("upsweep", "scan", "downsweep")


def cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "ng_autotune.json")


def _key(n_syn: int, n_nodes: int, max_delay: int) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    kb = max(n_nodes - 1, 0).bit_length() + int(max_delay).bit_length()
    return f"{dev}|n2^{max(0, math.ceil(math.log2(max(n_syn, 1))))}|keybits{kb}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(p + ".tmp", p)
    except OSError:
        pass


def tune(net, workload, candidates=CANDIDATES, reps: int = 2, use_cache: bool = True):
    """Return (radix_bits, sort_ranges) for this workload on this device."""
    key = _key(workload.n_syn, workload.n_nodes, workload.max_delay)
    cache = _load() if use_cache else {}
    if key in cache:
        return tuple(cache[key]["choice"])
    ctx = net.ctx
    args = [ng.call_args(c) for c in workload.calls]
    batch = [list(x) for x in zip(*args)]
    timings = {}
    for rb, ranges in candidates:
        ng.ng_set_tuning(ctx, rb, ranges)
        best = math.inf
        for _ in range(reps):
            ng.ng_reset(ctx)
            for n in workload.populations:
                ng.ng_create_nodes(ctx, n)
            ng.ng_connect_batch(ctx, *batch)
            ng.ng_sync(ctx)
            ng.ng_enable_timing(ctx, True)
            ng.ng_read_timing(ctx, reset=True)
            ng.ng_calibrate(ctx)
            t = ng.ng_read_timing(ctx, reset=True)
            ng.ng_enable_timing(ctx, False)
            best = min(best, sum(v[1] for k, v in t.items() if k in SORT_KERNELS))
        timings[f"{rb},{ranges}"] = best
    choice = min(candidates, key=lambda c: timings[f"{c[0]},{c[1]}"])
    ng.ng_reset(ctx)
    cache[key] = {"choice": list(choice), "sort_ms": timings}
    if use_cache:
        _save(cache)
    return tuple(choice)
