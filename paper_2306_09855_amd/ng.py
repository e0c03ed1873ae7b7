"""Python binding of the C ABI in include/ng.h (argument marshalling only).

Every function here has the name of the C entry point it wraps and raises
``NGError`` on a non-zero status.  All connection generation, sorting and
indexing runs in the HIP kernels of ``libng.so``; there is no fallback: if the
library is missing, ``lib()`` raises.

torch is imported before the library is loaded so that the process holds a
single HIP runtime (torch's); torch also supplies the device arena and the
stream (see ``arena_for``/``current_stream``).
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  (load torch's HIP runtime first)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libng.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ng.h")

NG_OK, NG_ERR_INVALID_ARG, NG_ERR_OOM, NG_ERR_UNSUPPORTED = 0, -1, -2, -3
NG_ERR_STATE, NG_ERR_TOO_LARGE, NG_ERR_DEVICE = -4, -5, -6

(NG_ONE_TO_ONE, NG_ALL_TO_ALL, NG_FIXED_INDEGREE, NG_FIXED_OUTDEGREE, NG_FIXED_TOTAL_NUMBER,
 NG_PAIRWISE_BERNOULLI) = range(6)
NG_CONST, NG_NORMAL, NG_UNIFORM_INT, NG_UNIFORM = range(4)

RULE_CODES = {"one_to_one": NG_ONE_TO_ONE, "all_to_all": NG_ALL_TO_ALL,
              "fixed_indegree": NG_FIXED_INDEGREE, "fixed_outdegree": NG_FIXED_OUTDEGREE,
              "fixed_total_number": NG_FIXED_TOTAL_NUMBER, "pairwise_bernoulli": NG_PAIRWISE_BERNOULLI}
DIST_CODES = {"const": NG_CONST, "normal": NG_NORMAL, "uniform_int": NG_UNIFORM_INT,
              "uniform": NG_UNIFORM}


class NGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ng status {status}: {msg}")
        self.status = status


class ng_range(ctypes.Structure):
    _fields_ = [("first", ctypes.c_uint32), ("n", ctypes.c_uint32)]


class ng_conn_spec(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("allow_autapses", ctypes.c_int32),
                ("allow_multapses", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("k_or_n", ctypes.c_uint64), ("p", ctypes.c_double)]


class ng_param(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class ng_syn_spec(ctypes.Structure):
    _fields_ = [("weight", ng_param), ("delay", ng_param)]


class ng_group(ctypes.Structure):
    """Node group: the range [first, first + n) when idx is NULL, else n indices at idx (device)."""
    _fields_ = [("first", ctypes.c_uint32), ("n", ctypes.c_uint32), ("idx", ctypes.c_void_p)]


class ng_schedule(ctypes.Structure):
    _fields_ = [("calibration", ctypes.c_int32), ("radix_bits", ctypes.c_int32), ("sort_ranges", ctypes.c_uint32),
                ("msd_tile", ctypes.c_uint32), ("gen_synapses_per_lane", ctypes.c_uint32),
                ("queued_calls", ctypes.c_uint32)]


class ng_config(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("h_ms", ctypes.c_float), ("reserved", ctypes.c_int32)]


class ng_conn_view(ctypes.Structure):
    _fields_ = [("n_conns", ctypes.c_uint64), ("n_groups", ctypes.c_uint64),
                ("block_size", ctypes.c_uint64), ("n_nodes", ctypes.c_uint32),
                ("n_blocks", ctypes.c_uint32), ("calibrated", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("block_base", ctypes.POINTER(ctypes.c_void_p)),
                ("group_ptr", ctypes.c_void_p), ("group_start", ctypes.c_void_p)]


class ng_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("records", ctypes.c_uint64)]


class ng_server_config(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_uint64), ("h_ms", ctypes.c_float), ("radix_bits", ctypes.c_int32),
                ("sort_ranges", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class ng_ticket_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("n_conns", ctypes.c_uint64),
                ("arrival_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64)]


class ng_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "launches", "packed_calls", "max_calls_per_launch",
                                                "calibrations", "sessions_opened", "peak_arena_bytes",
                                                "arena_used_bytes", "calibrate_packs", "max_sessions_per_pack",
                                                "scheduler_busy_ns", "host_launch_ns", "host_calibrate_ns")]


_lib = None


def lib():
    """Load libng.so (built by paper_2306_09855_amd/build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python paper_2306_09855_amd/build.py first")
        L = ctypes.CDLL(LIB_PATH)
        P, vp = ctypes.POINTER, ctypes.c_void_p
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        sig = {
            "ng_create": ([P(ng_config), vp, u64, vp, P(vp)], ctypes.c_int),
            "ng_destroy": ([vp], ctypes.c_int),
            "ng_create_nodes": ([vp, u32, P(ng_range)], ctypes.c_int),
            "ng_connect": ([vp, ng_range, ng_range, P(ng_conn_spec), P(ng_syn_spec), P(u32), P(u64),
                            P(u64)], ctypes.c_int),
            "ng_connect_groups": ([vp, ng_group, ng_group, P(ng_conn_spec), P(ng_syn_spec), vp, vp, P(u32),
                                   P(u64), P(u64)], ctypes.c_int),
            "ng_connect_batch": ([vp, u32, P(ng_range), P(ng_range), P(ng_conn_spec), P(ng_syn_spec),
                                  P(u64)], ctypes.c_int),
            "ng_calibrate": ([vp], ctypes.c_int),
            "ng_calibrate_many": ([P(vp), ctypes.c_uint32], ctypes.c_int),
            "ng_calibrate_noalloc": ([vp], ctypes.c_int),
            "ng_noalloc_scratch_bytes": ([], ctypes.c_uint64),
            "ng_sync": ([vp], ctypes.c_int),
            "ng_get_connections": ([vp, P(ng_conn_view)], ctypes.c_int),
            "ng_copy_connections": ([vp, u64, u64, vp, vp, vp, vp], ctypes.c_int),
            "ng_copy_group_index": ([vp, vp, vp], ctypes.c_int),
            "ng_set_tuning": ([vp, ctypes.c_int, u32], ctypes.c_int),
            "ng_set_calibration": ([vp, ctypes.c_int], ctypes.c_int),
            "ng_set_schedule": ([vp, P(ng_schedule)], ctypes.c_int),
            "ng_get_schedule": ([vp, P(ng_schedule)], ctypes.c_int),
            "ng_spikes_init": ([vp], ctypes.c_int),
            "ng_spikes_step": ([vp, vp, vp, u32, vp], ctypes.c_int),
            "ng_memory_stats": ([vp, P(u64), P(u64), P(u64)], ctypes.c_int),
            "ng_reset": ([vp], ctypes.c_int),
            "ng_set_seed": ([vp, u64], ctypes.c_int),
            "ng_enable_timing": ([vp, ctypes.c_int], ctypes.c_int),
            "ng_time_only": ([vp, ctypes.c_char_p], ctypes.c_int),
            "ng_read_timing": ([vp, P(ng_kernel_time), ctypes.c_int, P(ctypes.c_int), ctypes.c_int],
                               ctypes.c_int),
            "ng_graph_begin": ([vp, u64], ctypes.c_int),
            "ng_graph_end": ([vp, P(vp)], ctypes.c_int),
            "ng_graph_launch": ([vp, u64], ctypes.c_int),
            "ng_graph_destroy": ([vp], ctypes.c_int),
            "ng_server_create": ([P(ng_server_config), vp, u64, P(vp), ctypes.c_int, P(vp)], ctypes.c_int),
            "ng_server_destroy": ([vp], ctypes.c_int),
            "ng_session_open": ([vp, u64, P(vp)], ctypes.c_int),
            "ng_submit_create_nodes": ([vp, u32, P(ng_range), P(u64)], ctypes.c_int),
            "ng_submit_connect": ([vp, ng_range, ng_range, P(ng_conn_spec), P(ng_syn_spec), P(u64)],
                                  ctypes.c_int),
            "ng_submit_calibrate": ([vp, P(u64)], ctypes.c_int),
            "ng_submit_close": ([vp, P(u64)], ctypes.c_int),
            "ng_session_close": ([vp], ctypes.c_int),
            "ng_wait": ([vp, u64, ctypes.c_int64, P(ng_ticket_info)], ctypes.c_int),
            "ng_session_context": ([vp, P(vp)], ctypes.c_int),
            "ng_server_get_stats": ([vp, P(ng_server_stats)], ctypes.c_int),
            "ng_last_error": ([], ctypes.c_char_p),
            "ng_blocks_needed": ([u64, u64, u64, u64], u64),
            "ng_plan_count": ([u32, ng_range, ng_range, P(ng_conn_spec), P(ng_syn_spec), ctypes.c_float,
                               P(u64)], ctypes.c_int),
            "ng_calibration_plan": ([u64, u32, i32, u32, P(u32)], ctypes.c_int),
            "ng_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def declared_symbols() -> list:
    """Names of the functions include/ng.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ng_[a-z_]+)\s*\(", text)))


def _check(rc: int):
    if rc != NG_OK:
        raise NGError(rc, ng_last_error())


def _vp(x) -> ctypes.c_void_p:
    if x is None:
        return ctypes.c_void_p(0)
    if isinstance(x, torch.Tensor):
        return ctypes.c_void_p(x.data_ptr())
    if hasattr(x, "ctypes"):  # numpy
        return x.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(int(x))


# --- marshalling of workload descriptions ----------------------------------
def conn_spec(rule: str, k_or_n: int = 0, allow_autapses: int = 1, allow_multapses: int = 1,
              p: float = 0.0) -> ng_conn_spec:
    return ng_conn_spec(RULE_CODES[rule], allow_autapses, allow_multapses, 0, int(k_or_n), float(p))


def param(spec) -> ng_param:
    kind, a, b = (tuple(spec) + (0.0, 0.0))[:3]
    return ng_param(DIST_CODES[kind], 0, float(a), float(b))


def syn_spec(weight, delay) -> ng_syn_spec:
    return ng_syn_spec(param(weight), param(delay))


def call_args(call):
    """(src range, tgt range, conn spec, syn spec) of a workloads.Call."""
    return (ng_range(*call.src), ng_range(*call.tgt),
            conn_spec(call.rule, call.k_or_n, allow_autapses=int(getattr(call, "allow_autapses", 1)),
                      allow_multapses=int(getattr(call, "allow_multapses", 1)), p=float(getattr(call, "p", 0.0))),
            syn_spec(call.weight, call.delay))


# --- entry points ------------------------------------------------------------
def ng_version() -> str:
    return lib().ng_version().decode()


def ng_last_error() -> str:
    return lib().ng_last_error().decode()


def ng_blocks_needed(n_conns: int, n_new: int, block_size: int, n_blocks: int) -> int:
    return int(lib().ng_blocks_needed(n_conns, n_new, block_size, n_blocks))


def ng_plan_count(n_nodes: int, src: ng_range, tgt: ng_range, conn: ng_conn_spec, syn: ng_syn_spec,
                  h_ms: float = 0.1) -> int:
    out = ctypes.c_uint64()
    _check(lib().ng_plan_count(n_nodes, src, tgt, ctypes.byref(conn), ctypes.byref(syn), h_ms,
                               ctypes.byref(out)))
    return int(out.value)


def ng_calibration_plan(n_conns: int, n_nodes: int, max_delay: int, sort_ranges: int = 1024) -> dict:
    out = (ctypes.c_uint32 * 8)()
    _check(lib().ng_calibration_plan(n_conns, n_nodes, max_delay, sort_ranges, out))
    keys = ("msd", "b1", "b2", "b3", "narrow_a", "narrow_b", "wgs_c", "tpr")
    return {k: int(v) for k, v in zip(keys, out)}


def ng_create(cfg: ng_config, arena, arena_bytes: int, stream) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().ng_create(ctypes.byref(cfg), _vp(arena), arena_bytes, _vp(stream), ctypes.byref(h)))
    return h


def ng_destroy(ctx) -> None:
    _check(lib().ng_destroy(ctx))


def ng_create_nodes(ctx, n: int) -> ng_range:
    r = ng_range()
    _check(lib().ng_create_nodes(ctx, n, ctypes.byref(r)))
    return r


def ng_connect_groups(ctx, src: ng_group, tgt: ng_group, conn: ng_conn_spec, syn: ng_syn_spec,
                      weights=None, delays_ms=None):
    """ng_connect with node groups as index arrays and/or per-connection weights and delays
    (device pointers, as int addresses)."""
    cid, first, n = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().ng_connect_groups(ctx, src, tgt, ctypes.byref(conn), ctypes.byref(syn), _vp(weights),
                                   _vp(delays_ms), ctypes.byref(cid), ctypes.byref(first), ctypes.byref(n)))
    return int(cid.value), int(first.value), int(n.value)


def ng_connect(ctx, src: ng_range, tgt: ng_range, conn: ng_conn_spec, syn: ng_syn_spec):
    cid, first, n = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().ng_connect(ctx, src, tgt, ctypes.byref(conn), ctypes.byref(syn), ctypes.byref(cid),
                            ctypes.byref(first), ctypes.byref(n)))
    return int(cid.value), int(first.value), int(n.value)


def ng_connect_batch(ctx, srcs, tgts, conns, syns):
    n = len(srcs)
    S = (ng_range * n)(*srcs)
    T = (ng_range * n)(*tgts)
    C = (ng_conn_spec * n)(*conns)
    Y = (ng_syn_spec * n)(*syns)
    first = (ctypes.c_uint64 * n)()
    _check(lib().ng_connect_batch(ctx, n, S, T, C, Y, first))
    return [int(v) for v in first]


def ng_calibrate(ctx) -> None:
    _check(lib().ng_calibrate(ctx))


def ng_calibrate_noalloc(ctx) -> None:
    """ng_calibrate with its scratch in the library's fixed device region."""
    _check(lib().ng_calibrate_noalloc(ctx))


def ng_noalloc_scratch_bytes() -> int:
    return int(lib().ng_noalloc_scratch_bytes())


def ng_calibrate_many(ctxs) -> None:
    arr = (ctypes.c_void_p * len(ctxs))(*ctxs)
    _check(lib().ng_calibrate_many(arr, len(ctxs)))


def ng_sync(ctx) -> None:
    _check(lib().ng_sync(ctx))


def ng_get_connections(ctx) -> ng_conn_view:
    v = ng_conn_view()
    _check(lib().ng_get_connections(ctx, ctypes.byref(v)))
    return v


def ng_copy_connections(ctx, first: int, count: int, src=None, tgt=None, w=None, delay=None) -> None:
    _check(lib().ng_copy_connections(ctx, first, count, _vp(src), _vp(tgt), _vp(w), _vp(delay)))


def ng_copy_group_index(ctx, group_ptr=None, group_start=None) -> None:
    _check(lib().ng_copy_group_index(ctx, _vp(group_ptr), _vp(group_start)))


def ng_reset(ctx) -> None:
    _check(lib().ng_reset(ctx))


def ng_set_seed(ctx, seed: int) -> None:
    _check(lib().ng_set_seed(ctx, int(seed)))


def ng_enable_timing(ctx, on: bool = True) -> None:
    _check(lib().ng_enable_timing(ctx, 1 if on else 0))


def ng_time_only(ctx, name=None) -> None:
    """With timing on, events only around launches of this kernel name (None: all)."""
    _check(lib().ng_time_only(ctx, name.encode() if name else None))


def ng_read_timing(ctx, reset: bool = True, records: bool = False) -> dict:
    """{kernel name: (launches, total ms)} of the timed launches so far;
    with records=True, (launches, total ms, records processed)."""
    cap = 64
    arr = (ng_kernel_time * cap)()
    n = ctypes.c_int()
    _check(lib().ng_read_timing(ctx, arr, cap, ctypes.byref(n), 1 if reset else 0))
    rng = range(min(n.value, cap))
    if records:
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms), int(arr[i].records))
                for i in rng}
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in rng}


def ng_graph_begin(ctx, staging_bytes: int = 0) -> None:
    _check(lib().ng_graph_begin(ctx, staging_bytes))


def ng_graph_end(ctx) -> ctypes.c_void_p:
    g = ctypes.c_void_p()
    _check(lib().ng_graph_end(ctx, ctypes.byref(g)))
    return g


def ng_graph_launch(graph, seed: int) -> None:
    _check(lib().ng_graph_launch(graph, seed))


def ng_graph_destroy(graph) -> None:
    _check(lib().ng_graph_destroy(graph))


def ng_set_tuning(ctx, radix_bits: int, sort_ranges: int = 1024) -> None:
    _check(lib().ng_set_tuning(ctx, radix_bits, sort_ranges))


NG_CALIB_RADIX, NG_CALIB_COPASS, NG_CALIB_RADIX_LSD, NG_CALIB_RADIX_MSD = 0, 1, 2, 3
CALIBRATIONS = {"radix": NG_CALIB_RADIX, "copass": NG_CALIB_COPASS, "lsd": NG_CALIB_RADIX_LSD,
                "msd": NG_CALIB_RADIX_MSD}


def ng_set_calibration(ctx, algorithm) -> None:
    """Calibration algorithm: "radix" (default) or "copass" (in-place block sort)."""
    _check(lib().ng_set_calibration(ctx, CALIBRATIONS.get(algorithm, algorithm)))


SCHEDULE_KEYS = ("calibration", "radix_bits", "sort_ranges", "msd_tile", "gen_synapses_per_lane", "queued_calls")
QUEUED_CALLS_DEFAULT = 256


def ng_set_schedule(ctx, schedule: dict) -> None:
    """schedule: the fields of ng_schedule; calibration may be a name of CALIBRATIONS;
    queued_calls may be left out (256)."""
    cal = schedule["calibration"]
    sc = ng_schedule(CALIBRATIONS[cal] if isinstance(cal, str) else int(cal), int(schedule["radix_bits"]),
                     int(schedule["sort_ranges"]), int(schedule["msd_tile"]), int(schedule["gen_synapses_per_lane"]),
                     int(schedule.get("queued_calls", QUEUED_CALLS_DEFAULT)))
    _check(lib().ng_set_schedule(ctx, ctypes.byref(sc)))


def ng_get_schedule(ctx) -> dict:
    sc = ng_schedule()
    _check(lib().ng_get_schedule(ctx, ctypes.byref(sc)))
    names = {v: k for k, v in CALIBRATIONS.items()}
    out = {k: int(getattr(sc, k)) for k in SCHEDULE_KEYS}
    out["calibration"] = names.get(out["calibration"], out["calibration"])
    return out


def ng_memory_stats(ctx):
    u, p, f = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().ng_memory_stats(ctx, ctypes.byref(u), ctypes.byref(p), ctypes.byref(f)))
    return int(u.value), int(p.value), int(f.value)


# --- serving form -------------------------------------------------------------------
def ng_server_create(cfg: ng_server_config, arena, arena_bytes: int, streams) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(streams))(*[int(x) for x in streams])
    h = ctypes.c_void_p()
    _check(lib().ng_server_create(ctypes.byref(cfg), _vp(arena), arena_bytes, arr, len(streams),
                                  ctypes.byref(h)))
    return h


def ng_server_destroy(server) -> None:
    _check(lib().ng_server_destroy(server))


def ng_session_open(server, seed: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().ng_session_open(server, seed, ctypes.byref(h)))
    return h


def ng_submit_create_nodes(session, n: int):
    r, t = ng_range(), ctypes.c_uint64()
    _check(lib().ng_submit_create_nodes(session, n, ctypes.byref(r), ctypes.byref(t)))
    return (r.first, r.n), int(t.value)


def ng_submit_connect(session, src: ng_range, tgt: ng_range, conn: ng_conn_spec, syn: ng_syn_spec) -> int:
    t = ctypes.c_uint64()
    _check(lib().ng_submit_connect(session, src, tgt, ctypes.byref(conn), ctypes.byref(syn), ctypes.byref(t)))
    return int(t.value)


def ng_submit_calibrate(session) -> int:
    t = ctypes.c_uint64()
    _check(lib().ng_submit_calibrate(session, ctypes.byref(t)))
    return int(t.value)


def ng_submit_close(session) -> int:
    t = ctypes.c_uint64()
    _check(lib().ng_submit_close(session, ctypes.byref(t)))
    return int(t.value)


def ng_session_close(session) -> None:
    _check(lib().ng_session_close(session))


def ng_wait(server, ticket: int, timeout_ns: int = -1) -> ng_ticket_info:
    info = ng_ticket_info()
    _check(lib().ng_wait(server, ticket, timeout_ns, ctypes.byref(info)))
    return info


def ng_session_context(session) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().ng_session_context(session, ctypes.byref(h)))
    return h


def ng_server_get_stats(server) -> dict:
    st = ng_server_stats()
    _check(lib().ng_server_get_stats(server, ctypes.byref(st)))
    return {n: int(getattr(st, n)) for n, _ in ng_server_stats._fields_}


# --- torch plumbing: device memory and streams ----------------------------------
def arena_for(nbytes: int, device: str = "cuda") -> torch.Tensor:
    """A device buffer the context carves its allocations from."""
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def current_stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def group(g) -> ng_group:
    """ng_group from (first, n), or from a device tensor of node indices."""
    if isinstance(g, ng_group):
        return g
    if isinstance(g, torch.Tensor):
        if not g.is_cuda or g.dtype not in (torch.int32, torch.uint32) or not g.is_contiguous():
            raise ValueError("index arrays are contiguous 32-bit device tensors")
        return ng_group(0, g.numel(), g.data_ptr())
    return ng_group(int(g[0]), int(g[1]), None)


def ng_spikes_init(ctx) -> None:
    """Spike buffers over the calibrated connections (Sec. 2.3); synchronizes."""
    _check(lib().ng_spikes_init(ctx))


def ng_spikes_step(ctx, nodes, mult, n: int, input) -> None:
    """One step: queued spikes advance and deliver input[t] += w * m; then nodes emit."""
    _check(lib().ng_spikes_step(ctx, _vp(nodes), _vp(mult), n, _vp(input)))
