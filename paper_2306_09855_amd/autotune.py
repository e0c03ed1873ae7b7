"""Autotuner for a context's kernel schedule (ng_schedule).

For a workload it times, on this device, the generation kernels for each
number of synapses per lane and the calibration kernels for each calibration
form with its tile, digit and range settings, keeps the fastest of each when
it beats the default schedule by at least MARGIN (closer than that, the
timings' noise would decide, and the default stays), and caches the choice
as JSON per device, keyed by the connection count and the
key density (both rounded to powers of two) and the key width.  The
arithmetic never depends on the schedule -- only the speed does -- which the
tests check by building under the chosen and the default schedule.

Search space:
  gen_synapses_per_lane   4, 8, 16                    (generation kernels)
  most-significant-digit  msd_tile 16384 / 10240 x sort_ranges 512 / 1024 / 2048
                          (the second scatter takes three times as many ranges)
  LSD                     radix_bits 8 / 9 x sort_ranges 512 / 1024 / 2048
(the MSD form only where it applies: keys of at most 27 bits).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import ng

DEFAULT = {"calibration": "radix", "radix_bits": 9, "sort_ranges": 1024, "msd_tile": 16384,
           "gen_synapses_per_lane": 4, "queued_calls": 256}
GEN_SPL = (4, 8, 16)
MARGIN = 0.02  # a candidate replaces the default only when this much faster
RANGES = (512, 1024, 2048)
GEN_KERNELS = ("generate", "generate_batch")


def cache_path() -> str:
    p = os.environ.get("NG_AUTOTUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "ng_autotune.json")


def _key(workload, batched: bool) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    dbits = int(workload.max_delay).bit_length()
    kb = max(workload.n_nodes - 1, 0).bit_length() + dbits
    n = max(workload.n_syn, 1)
    density = n / max(workload.n_nodes << dbits, 1)
    return (f"{dev}|n2^{math.ceil(math.log2(n))}|keybits{kb}|density2^{round(math.log2(density))}"
            f"|{'batched' if batched else 'plain'}")


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def calibration_candidates(workload) -> list:
    plan = ng.ng_calibration_plan(workload.n_syn, workload.n_nodes, workload.max_delay)
    cands = []
    if plan["msd"] >= 1:
        tiles = (16384, 10240) if plan["narrow_a"] and plan["b2"] else (16384,)
        cands += [{"calibration": "msd", "msd_tile": t, "sort_ranges": r, "radix_bits": 9}
                  for t in tiles for r in RANGES]
    cands += [{"calibration": "lsd", "msd_tile": 16384, "sort_ranges": r, "radix_bits": b}
              for b in (8, 9) for r in RANGES]
    return cands


def _build(ctx, workload, args, batch, batched):
    ng.ng_reset(ctx)
    for n in workload.populations:
        ng.ng_create_nodes(ctx, n)
    if batched:
        ng.ng_connect_batch(ctx, *batch)
    else:
        for a in args:
            ng.ng_connect(ctx, *a)


def _timed(ctx, fn, names=None) -> float:
    """Device milliseconds of the kernels fn launches (all of them, or those named)."""
    ng.ng_sync(ctx)
    ng.ng_enable_timing(ctx, True)
    ng.ng_read_timing(ctx, reset=True)
    fn()
    ng.ng_sync(ctx)
    t = ng.ng_read_timing(ctx, reset=True)
    ng.ng_enable_timing(ctx, False)
    return sum(v[1] for k, v in t.items() if names is None or k in names)


def tune(net, workload, batched: bool = False, reps: int = 3, use_cache: bool = True):
    """The schedule for this workload on this device, as a dict of
    ng_schedule fields (per field group, the fastest candidate where it beats
    the default by MARGIN, else the default), and whether it came from the
    cache.  The context is left reset, with its previous schedule."""
    key = _key(workload, batched)
    path = cache_path()
    cache = _load(path) if use_cache else {}
    if key in cache:
        return dict(cache[key]["choice"]), True
    ctx = net.ctx
    saved = ng.ng_get_schedule(ctx)
    args = [ng.call_args(c) for c in workload.calls]
    batch = [list(x) for x in zip(*args)]
    gen_ms = {}
    for spl in GEN_SPL:
        ng.ng_set_schedule(ctx, {**DEFAULT, "gen_synapses_per_lane": spl})
        gen_ms[spl] = min(_timed(ctx, lambda: _build(ctx, workload, args, batch, batched), GEN_KERNELS)
                          for _ in range(reps))
    best_spl = min(GEN_SPL, key=lambda s: gen_ms[s])
    if gen_ms[best_spl] > (1 - MARGIN) * gen_ms[DEFAULT["gen_synapses_per_lane"]]:
        best_spl = DEFAULT["gen_synapses_per_lane"]

    def calibrate_ms(sched):
        ng.ng_set_schedule(ctx, sched)
        best = math.inf
        for _ in range(reps):
            _build(ctx, workload, args, batch, batched)
            best = min(best, _timed(ctx, lambda: ng.ng_calibrate(ctx)))
        return best

    default_ms = calibrate_ms({**DEFAULT, "gen_synapses_per_lane": best_spl})
    cal_ms = {}
    for cand in calibration_candidates(workload):
        cal_ms[json.dumps(cand, sort_keys=True)] = calibrate_ms({**DEFAULT, **cand, "gen_synapses_per_lane": best_spl})
    best_key = min(cal_ms, key=cal_ms.get)
    best_cal = json.loads(best_key) if cal_ms[best_key] <= (1 - MARGIN) * default_ms else {}
    choice = {**DEFAULT, **best_cal, "gen_synapses_per_lane": best_spl}
    ng.ng_reset(ctx)
    ng.ng_set_schedule(ctx, saved)
    cache[key] = {"choice": choice, "generate_ms": {str(k): v for k, v in gen_ms.items()},
                  "calibrate_ms": cal_ms, "default_calibrate_ms": default_ms}
    if use_cache:
        _save(path, cache)
    return choice, False
