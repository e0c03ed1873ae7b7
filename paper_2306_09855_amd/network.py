"""A thin convenience wrapper over the C ABI: one context on a torch arena.

Everything it does is marshalling: nodes, Connect calls and calibration go
straight to libng.so; ``fetch`` copies the device result into host or device
buffers the caller can inspect.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ng


def arena_bytes_for(n_syn: int, n_nodes: int, max_delay: int = 63, block_size: int = 1 << 24,
                    radix_bits: int = 8, slack: float = 1.15) -> int:
    """Arena size that holds n_syn connections through one calibration."""
    blocks = -(-max(n_syn, 1) // block_size)
    store = 14 * block_size * blocks                 # creation-order blocks
    sorted_store = store                             # calibrated blocks
    scratch = 2 * 12 * n_syn                         # two key/payload buffers (3+ passes)
    status = 8 * (1 << radix_bits) * (n_syn // 4096 + 1)   # digit counts and tables (upper bound)
    index = 4 * (n_nodes + 1) * 3 + 4 * (min(n_syn, n_nodes * max_delay) + 1) + 4 * (n_syn // 4096 + 8)
    total = int((store + sorted_store + scratch + status + index) * slack) + (64 << 20)
    return (total + 4095) // 4096 * 4096


class Network:
    def __init__(self, seed: int, h: float = 0.1, block_size: int = 0, arena_bytes: int = 1 << 30,
                 stream: int | None = None, device: str = "cuda"):
        self.arena_bytes = int(arena_bytes)
        self.arena = ng.arena_for(self.arena_bytes, device)
        self.stream = ng.current_stream() if stream is None else stream
        cfg = ng.ng_config(int(block_size), int(seed), float(h), 0)
        self.ctx = ng.ng_create(cfg, self.arena, self.arena_bytes, self.stream)

    # -- construction ---------------------------------------------------------
    def create(self, n: int):
        r = ng.ng_create_nodes(self.ctx, int(n))
        return r.first, r.n

    def connect(self, call):
        return ng.ng_connect(self.ctx, *ng.call_args(call))

    def connect_batch(self, calls):
        args = [ng.call_args(c) for c in calls]
        return ng.ng_connect_batch(self.ctx, [a[0] for a in args], [a[1] for a in args],
                                   [a[2] for a in args], [a[3] for a in args])

    def calibrate(self):
        ng.ng_calibrate(self.ctx)

    def sync(self):
        ng.ng_sync(self.ctx)

    def tune(self, radix_bits: int, sort_ranges: int = 1024):
        ng.ng_set_tuning(self.ctx, radix_bits, sort_ranges)

    def connect_groups(self, call, src, tgt, weights=None, delays_ms=None):
        """A Connect call whose groups may be index tensors (device, int32) and whose weights
        / delays (ms) may be per-connection device tensors (float32); the rule, K/N and
        distributions come from `call`."""
        conn = ng.conn_spec(call.rule, call.k_or_n, allow_autapses=int(getattr(call, "allow_autapses", 1)))
        return ng.ng_connect_groups(self.ctx, ng.group(src), ng.group(tgt), conn,
                                    ng.syn_spec(call.weight, call.delay), weights, delays_ms)

    def spikes_init(self):
        ng.ng_spikes_init(self.ctx)

    def spikes_step(self, nodes, input, mult=None):
        """One simulation step (Sec. 2.3): nodes (device int32/uint32 tensor) emit after the
        queued spikes are delivered into input (device float32 tensor, accumulated)."""
        n = 0 if nodes is None else nodes.numel()
        ng.ng_spikes_step(self.ctx, nodes if n else None, mult, n, input)

    def set_calibration(self, algorithm: str):
        """"radix" (default) or "copass": the in-place block sort of the appendix."""
        ng.ng_set_calibration(self.ctx, algorithm)

    def build(self, workload, batched: bool = False, calibrate: bool = True):
        for n in workload.populations:
            self.create(n)
        if batched:
            self.connect_batch(workload.calls)
        else:
            for c in workload.calls:
                self.connect(c)
        if calibrate:
            self.calibrate()
        return self

    # -- read back -----------------------------------------------------------------
    def view(self):
        return ng.ng_get_connections(self.ctx)

    def fetch(self, first: int = 0, count: int | None = None, device: bool = False):
        v = self.view()
        n = v.n_conns - first if count is None else count
        if device:
            mk = lambda dt: torch.empty(n, dtype=dt, device="cuda")  # noqa: E731
            out = dict(src=mk(torch.int32), tgt=mk(torch.int32), w=mk(torch.float32), delay=mk(torch.int16))
        else:
            out = dict(src=np.empty(n, np.uint32), tgt=np.empty(n, np.uint32), w=np.empty(n, np.float32),
                       delay=np.empty(n, np.int16))
        if n:
            ng.ng_copy_connections(self.ctx, first, n, out["src"], out["tgt"], out["w"], out["delay"])
        return out

    def group_index(self):
        v = self.view()
        gp = np.empty(v.n_nodes + 1, np.uint32)
        gs = np.empty(v.n_groups + 1, np.uint32)
        ng.ng_copy_group_index(self.ctx, gp, gs)
        return gp, gs

    def memory_stats(self):
        return ng.ng_memory_stats(self.ctx)

    def close(self):
        if self.ctx is not None:
            ng.ng_destroy(self.ctx)
            self.ctx = None
            self.arena = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def calibrate_many(nets) -> None:
    """Calibrate several networks in shared launches (ng_calibrate_many); the
    first network's stream runs them and its arena holds the shared scratch."""
    ng.ng_calibrate_many([n.ctx for n in nets])


class Graph:
    """A captured build (batched form) that can be replayed with any seed."""

    def __init__(self, net: Network, build_fn):
        ng.ng_graph_begin(net.ctx)
        try:
            build_fn(net)
        except Exception:
            ng.ng_graph_destroy(ng.ng_graph_end(net.ctx))
            raise
        self.handle = ng.ng_graph_end(net.ctx)

    def launch(self, seed: int):
        ng.ng_graph_launch(self.handle, seed)

    def close(self):
        if self.handle is not None:
            ng.ng_graph_destroy(self.handle)
            self.handle = None
