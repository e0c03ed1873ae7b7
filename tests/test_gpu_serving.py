"""Serving form: sessions submitted from several client threads, admitted by
free arena memory, packed into shared launches.  Each session's result must
equal the same calls built alone (same seed, same order) and the oracle."""
import threading

import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W
from parity import check_calibrated

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd import ng  # noqa: E402
from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402

B = 1 << 16


def _server(arena_bytes, n_streams=3):
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    arena = ng.arena_for(arena_bytes)
    srv = ng.ng_server_create(ng.ng_server_config(B, 0.1, 0, 0, 0), arena, arena_bytes,
                              [s.cuda_stream for s in streams])
    return srv, arena, streams


def _session_workloads():
    out = []
    for i in range(6):
        wl = W.batch_mixed(n_calls=12 + 3 * i, n_nodes=20_000 + 5_000 * i, lo_exp=1.0, hi_exp=4.3, gen_seed=100 + i)
        wl.seed = 1000 + i
        out.append(wl)
    return out


def _run_session(srv, wl, tickets):
    ss = ng.ng_session_open(srv, wl.seed)
    for n in wl.populations:
        _, t = ng.ng_submit_create_nodes(ss, n)
        tickets.append(t)
    for c in wl.calls:
        tickets.append(ng.ng_submit_connect(ss, *ng.call_args(c)))
    tickets.append(ng.ng_submit_calibrate(ss))
    return ss


def _fetch_session(ss, n_nodes):
    ctx = ng.ng_session_context(ss)
    v = ng.ng_get_connections(ctx)
    n = v.n_conns
    out = dict(src=np.empty(n, np.uint32), tgt=np.empty(n, np.uint32), w=np.empty(n, np.float32),
               delay=np.empty(n, np.int16))
    if n:
        ng.ng_copy_connections(ctx, 0, n, out["src"], out["tgt"], out["w"], out["delay"])
    gp = np.empty(v.n_nodes + 1, np.uint32)
    gs = np.empty(v.n_groups + 1, np.uint32)
    ng.ng_copy_group_index(ctx, gp, gs)
    return out, gp, gs


def _alone(wl):
    with Network(wl.seed, wl.h, B, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B)) as net:
        net.build(wl)
        out = net.fetch()
        gp, gs = net.group_index()
    return out, gp, gs


def test_served_equals_alone_and_oracle():
    wls = _session_workloads()
    srv, arena, streams = _server(1 << 30)
    sessions, tickets = [None] * len(wls), [[] for _ in wls]

    def client(idx):
        for i in idx:
            sessions[i] = _run_session(srv, wls[i], tickets[i])

    threads = [threading.Thread(target=client, args=(list(range(k, len(wls), 3)),)) for k in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for i, wl in enumerate(wls):
        for t in tickets[i]:
            info = ng.ng_wait(srv, t)
            assert info.status == 0, (i, info.status)
            assert info.done_ns >= info.admit_ns >= info.arrival_ns
    stats = ng.ng_server_get_stats(srv)
    assert stats["calibrations"] == len(wls)
    for i, wl in enumerate(wls):
        served = _fetch_session(sessions[i], wl.n_nodes)
        alone = _alone(wl)
        for k in ("src", "tgt", "delay", "w"):
            assert np.array_equal(served[0][k], alone[0][k]), (i, k)
        assert np.array_equal(served[1], alone[1]) and np.array_equal(served[2], alone[2])
        if i == 0:
            ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
            check_calibrated(served[0], served[1], served[2], ref, wl.calls)
    for ss in sessions:
        ng.ng_wait(srv, ng.ng_submit_close(ss))
    ng.ng_server_destroy(srv)


def test_admission_waits_for_memory():
    # Session a (1e5 synapses) peaks near 5.2 MB while it calibrates and then
    # holds about 2 MB.  Session b's one Connect needs 7 blocks of 2^16
    # connections (6.4 MB): in a 7.5 MB arena it waits until a closes, then
    # runs.  b's calibration would need another 6.4 MB of sorted blocks plus
    # scratch, more than the arena can ever give it, so it fails at once.
    wl = W.two_pop_indegree(scale=1.0)
    srv, arena, streams = _server(7_500_000 // 256 * 256, n_streams=2)
    a = ng.ng_session_open(srv, 1)
    b = ng.ng_session_open(srv, 2)
    ta = [ng.ng_submit_create_nodes(a, n)[1] for n in wl.populations]
    ta += [ng.ng_submit_connect(a, *ng.call_args(c)) for c in wl.calls]
    ta.append(ng.ng_submit_calibrate(a))
    tb0 = ng.ng_submit_create_nodes(b, 2000)[1]
    tb = ng.ng_submit_connect(b, ng.ng_range(0, 2000), ng.ng_range(0, 2000),
                              ng.conn_spec("fixed_total_number", 400_000),
                              ng.syn_spec(("const", 1.0), ("const", 1.0)))
    for t in ta:
        assert ng.ng_wait(srv, t).status == 0
    assert ng.ng_wait(srv, tb0).status == 0
    # b's connect cannot fit while a holds its connections
    with pytest.raises(ng.NGError) as e:
        ng.ng_wait(srv, tb, timeout_ns=200_000_000)
    assert e.value.status == ng.NG_ERR_STATE
    ng.ng_session_close(a)  # submits the close and waits for it
    info = ng.ng_wait(srv, tb)
    assert info.status == 0 and info.n_conns == 400_000
    assert ng.ng_wait(srv, ng.ng_submit_calibrate(b)).status == ng.NG_ERR_OOM
    ng.ng_server_destroy(srv)


def test_hopeless_and_invalid_requests():
    srv, arena, streams = _server(32 << 20, n_streams=1)
    # another session holds arena memory, idle: a request larger than the
    # whole arena must still fail at once instead of waiting for it
    other = ng.ng_session_open(srv, 6)
    ng.ng_wait(srv, ng.ng_submit_create_nodes(other, 100)[1])
    assert ng.ng_wait(srv, ng.ng_submit_connect(other, ng.ng_range(0, 100), ng.ng_range(0, 100),
                                                ng.conn_spec("all_to_all"),
                                                ng.syn_spec(("const", 1.0), ("const", 1.0)))).status == 0
    s = ng.ng_session_open(srv, 5)
    (first, n), t0 = ng.ng_submit_create_nodes(s, 100)
    bad = ng.ng_submit_connect(s, ng.ng_range(0, 100), ng.ng_range(0, 99), ng.conn_spec("one_to_one"),
                               ng.syn_spec(("const", 1.0), ("const", 1.0)))
    big = ng.ng_submit_connect(s, ng.ng_range(0, 100), ng.ng_range(0, 100),
                               ng.conn_spec("fixed_total_number", 50_000_000),
                               ng.syn_spec(("const", 1.0), ("const", 1.0)))
    ok = ng.ng_submit_connect(s, ng.ng_range(0, 100), ng.ng_range(0, 100), ng.conn_spec("all_to_all"),
                              ng.syn_spec(("const", 1.0), ("const", 1.0)))
    assert ng.ng_wait(srv, t0).status == 0
    assert ng.ng_wait(srv, bad).status == ng.NG_ERR_INVALID_ARG
    assert ng.ng_wait(srv, big).status == ng.NG_ERR_OOM
    info = ng.ng_wait(srv, ok)
    assert info.status == 0 and info.n_conns == 10_000
    ng.ng_server_destroy(srv)   # closes the open session
