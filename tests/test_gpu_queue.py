"""ng_connect's queue: Connect calls below 2^24 synapses wait in the context
and go out together as one generation launch when a call needs their
connections.  The arrays never depend on it: every case compares the build
with the same build whose queue is off (queued_calls = 0: one launch per
call) bit for bit, and the small builds with the oracle, and each case goes
through one of the points that launch the queue (calibrate, sync and the
reads that synchronize, a batch, node arrays, pairwise_bernoulli, a lower queue
bound, the fixed-scratch calibration) or drops it (reset); a large call
launches at once and leaves the queue waiting."""
import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W
from parity import check_calibrated, check_creation_order

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd import ng  # noqa: E402
from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402

SEED = 77
N_NODES = 40_000


def _small_calls():
    w, d = ("normal", 0.5, 0.05), ("uniform_int", 1, 30)
    return [
        W.Call("fixed_total_number", (0, 3000), (1000, 5000), 70_001, w, d),
        W.Call("fixed_indegree", (500, 2000), (0, 700), 33, ("uniform", -1.0, 1.0), ("uniform", 0.1, 3.0)),
        W.Call("one_to_one", (10, 999), (2000, 999), 0, ("const", 1.5), ("const", 0.7)),
        W.Call("fixed_outdegree", (7000, 301), (0, 9000), 17, w, d),
        W.Call("all_to_all", (100, 37), (300, 41), 0, w, d),
        W.Call("fixed_total_number", (20_000, 5), (20_000, 5), 3, w, d),
    ]


def _set_queue(net, n):
    ng.ng_set_schedule(net.ctx, {**ng.ng_get_schedule(net.ctx), "queued_calls": n})
    assert ng.ng_get_schedule(net.ctx)["queued_calls"] == n


def _net(n_syn, block=1 << 16):
    return Network(SEED, 0.1, block, arena_bytes_for(max(n_syn, 1), N_NODES, 63, block))


def _build(calls, queue, between=None, block=1 << 16):
    """Create the nodes, connect the calls (between(net, i) after call i),
    read the creation order, calibrate, read the calibrated arrays."""
    n_syn = sum(c.n_syn() for c in calls)
    with _net(n_syn, block) as net:
        _set_queue(net, queue)
        net.create(N_NODES)
        for i, c in enumerate(calls):
            net.connect(c)
            if between:
                between(net, i)
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
        net.sync()
    return created, out, gp, gs


def _same(a, b):
    for x, y in zip(a[:2], b[:2]):
        for k in ("src", "tgt", "delay"):
            assert np.array_equal(x[k], y[k]), k
        assert np.array_equal(x["w"].view(np.uint32), y["w"].view(np.uint32))
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


@pytest.mark.parametrize("queue", [256, 3, 1])
def test_queue_equals_one_launch_per_call_and_oracle(queue):
    calls = _small_calls() * 3  # 18 calls: several launches for the small bounds
    ref = oracle.build_network(SEED, 0.1, N_NODES, calls)
    got = _build(calls, queue)
    check_creation_order(got[0], ref, calls)
    check_calibrated(got[1], got[2], got[3], ref, calls)
    _same(got, _build(calls, 0))


def test_large_call_between_queued_calls():
    # a call of 2^24 + 3 synapses launches at once; the queued calls before it
    # wait and go out after it, with the ones queued later, at the calibration
    big = W.Call("fixed_total_number", (0, N_NODES), (0, N_NODES), (1 << 24) + 3,
                 ("normal", 0.5, 0.05), ("uniform_int", 1, 30))
    calls = _small_calls()[:3] + [big] + _small_calls()[3:]
    _same(_build(calls, 256, block=1 << 22), _build(calls, 0, block=1 << 22))


def test_reads_and_syncs_launch_the_queue():
    # creation order read after every call (ng_copy_connections synchronizes)
    calls = _small_calls()
    ref = oracle.build_network(SEED, 0.1, N_NODES, calls)
    seen = []

    def read(net, i):
        v = net.view()
        assert v.n_conns == sum(c.n_syn() for c in calls[: i + 1])
        seen.append(net.fetch())

    got = _build(calls, 256, between=read)
    check_creation_order(got[0], ref, calls)
    check_calibrated(got[1], got[2], got[3], ref, calls)
    for i, part in enumerate(seen):
        n = part["src"].size
        assert np.array_equal(part["src"], got[0]["src"][:n]), i


def test_lower_bound_launches_what_the_queue_holds():
    calls = _small_calls()

    def lower(net, i):
        if i == 3:  # four calls queued; the new bound of 2 launches them
            _set_queue(net, 2)

    _same(_build(calls, 256, between=lower), _build(calls, 0))


def test_reset_drops_the_queue():
    calls = _small_calls()
    n_syn = sum(c.n_syn() for c in calls)
    with _net(2 * n_syn) as net:
        net.create(N_NODES)
        for c in calls[::-1]:  # queued, then discarded
            net.connect(c)
        ng.ng_reset(net.ctx)
        net.create(N_NODES)
        for c in calls:
            net.connect(c)
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    ref = oracle.build_network(SEED, 0.1, N_NODES, calls)
    check_creation_order(created, ref, calls)
    check_calibrated(out, gp, gs, ref, calls)


def test_batch_arrays_and_pairwise_after_queued_calls():
    calls = _small_calls()
    pw = W.Call("all_to_all", (3000, 200), (100, 300), 0, ("normal", 0.5, 0.05), ("uniform_int", 1, 30))
    pw_spec = ng.conn_spec("pairwise_bernoulli", 0, p=0.25)

    def build(queue):
        with _net(400_000) as net:
            _set_queue(net, queue)
            net.create(N_NODES)
            for c in calls[:2]:
                net.connect(c)
            net.connect_batch(calls[2:4])  # launches the two queued calls first
            net.connect(calls[4])
            idx = torch.arange(5000, 5100, dtype=torch.int32, device="cuda").flip(0).contiguous()
            net.connect_groups(calls[5], idx, calls[5].tgt)  # node array: synchronizes
            net.connect(calls[0])
            ng.ng_connect(net.ctx, ng.ng_range(*pw.src), ng.ng_range(*pw.tgt), pw_spec,
                          ng.syn_spec(pw.weight, pw.delay))  # counts on the device: synchronizes
            net.connect(calls[1])
            created = net.fetch()
            net.calibrate()
            out = net.fetch()
            gp, gs = net.group_index()
            net.sync()
        return created, out, gp, gs

    _same(build(256), build(0))


def test_fixed_scratch_calibration_after_queued_calls():
    calls = _small_calls()
    n_syn = sum(c.n_syn() for c in calls)
    ref = oracle.build_network(SEED, 0.1, N_NODES, calls)
    with _net(n_syn) as net:
        net.create(N_NODES)
        for c in calls:
            net.connect(c)
        ng.ng_calibrate_noalloc(net.ctx)  # launches the queue one call at a time
        out = net.fetch()
        gp, gs = net.group_index()
    check_calibrated(out, gp, gs, ref, calls)
