"""Packed calibration (ng_calibrate_many): contexts calibrated together, each
one a segment of the same sort and group-index launches, must each hold
exactly what ng_calibrate gives it alone -- and what the oracle gives."""
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
from paper_2306_09855_amd.network import Network, arena_bytes_for, calibrate_many  # noqa: E402

B = 1 << 16


def _mixed_workloads():
    """Key widths that give 1, 2, 3 and 4 digit passes, an empty context and
    several calls per context."""
    tiny = W.Workload("tiny", 77, [40], [W.Call("all_to_all", (0, 40), (0, 40), 0, ("const", 1.0),
                                                ("uniform_int", 1, 3))])           # 6+2 bits: 1 pass
    empty = W.Workload("empty", 78, [1000], [])
    c1 = W.two_pop_indegree(scale=1.0)                                            # 11+5 bits: 2 passes
    mc = W.microcircuit(scale=0.05)                                               # 12+5 bits: 3 passes
    mixed = W.batch_mixed(n_calls=24, n_nodes=300_000, lo_exp=1.0, hi_exp=5.2, gen_seed=7)  # 19+6: 4 passes
    mixed.seed = 4242
    return [c1, tiny, mc, empty, mixed]


def _net(wl, extra=0, stream=None):
    return Network(wl.seed, wl.h, B, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B) + extra,
                   stream=stream)


def _result(net):
    out = net.fetch()
    gp, gs = net.group_index()
    return out, gp, gs


def _alone(wl, radix_bits=8):
    with _net(wl) as net:
        net.tune(radix_bits)
        net.build(wl)
        return _result(net)


def _same(a, b, tag):
    for k in ("src", "tgt", "delay", "w"):
        assert np.array_equal(a[0][k], b[0][k]), (tag, k)
    assert np.array_equal(a[1], b[1]), (tag, "group_ptr")
    assert np.array_equal(a[2], b[2]), (tag, "group_start")


def test_packed_equals_alone_and_oracle():
    wls = _mixed_workloads()
    streams = [torch.cuda.Stream() for _ in wls]
    radix = [8, 8, 9, 8, 8]   # the 9-bit context shares a pack with 8-bit ones (2 passes each)
    nets = [_net(wl, extra=(256 << 20) if i == 0 else 0, stream=streams[i].cuda_stream)
            for i, wl in enumerate(wls)]
    try:
        for net, wl, rb in zip(nets, wls, radix):
            net.tune(rb)
            net.build(wl, calibrate=False)
        calibrate_many(nets)
        for i, (net, wl) in enumerate(zip(nets, wls)):
            got = _result(net)
            _same(got, _alone(wl, radix[i]), wl.name)
            ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
            check_calibrated(got[0], got[1], got[2], ref, wl.calls)
    finally:
        for net in nets:
            net.close()


def test_many_small_contexts_one_stream():
    # 48 segments: the range, tile and ptr-block tables are exercised across
    # many segments; a shared stream needs no cross-stream ordering
    wls = []
    for i in range(48):
        wl = W.batch_mixed(n_calls=3 + i % 5, n_nodes=2_000 + 397 * i, lo_exp=1.0, hi_exp=3.7, gen_seed=300 + i)
        wl.seed = 9000 + i
        wls.append(wl)
    nets = [_net(wl, extra=(128 << 20) if i == 0 else 0) for i, wl in enumerate(wls)]
    try:
        for net, wl in zip(nets, wls):
            net.build(wl, calibrate=False)
        calibrate_many(nets)
        for net, wl in zip(nets, wls):
            got = _result(net)
            ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
            check_calibrated(got[0], got[1], got[2], ref, wl.calls)
    finally:
        for net in nets:
            net.close()


def test_packed_connect_after_and_skip_calibrated():
    wls = _mixed_workloads()[:3]
    nets = [_net(wl, extra=(64 << 20)) for wl in wls]
    try:
        for net, wl in zip(nets, wls):
            net.build(wl, calibrate=False)
        calibrate_many(nets)
        # more connections into one context only: the others are skipped
        extra = W.Call("fixed_total_number", (0, wls[0].n_nodes), (0, wls[0].n_nodes), 5_000,
                       ("normal", 0.5, 0.05), ("uniform_int", 1, 20))
        nets[0].connect(extra)
        before = [_result(n) for n in nets[1:]]
        calibrate_many(nets)
        for net, b in zip(nets[1:], before):
            _same(_result(net), b, "skipped")
        calls = wls[0].calls + [extra]
        ref = oracle.build_network(wls[0].seed, wls[0].h, wls[0].n_nodes, calls)
        got = _result(nets[0])
        check_calibrated(got[0], got[1], got[2], ref, calls)
    finally:
        for net in nets:
            net.close()


def test_packed_argument_errors():
    wl = W.two_pop_indegree(scale=0.2)
    a, b = _net(wl), _net(wl)
    other = Network(wl.seed, wl.h, 1 << 17, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, 1 << 17))
    try:
        for n in (a, b, other):
            n.build(wl, calibrate=False)
        with pytest.raises(ng.NGError) as e:
            ng.ng_calibrate_many([a.ctx, a.ctx])
        assert e.value.status == ng.NG_ERR_INVALID_ARG
        with pytest.raises(ng.NGError) as e:
            ng.ng_calibrate_many([a.ctx, other.ctx])
        assert e.value.status == ng.NG_ERR_INVALID_ARG
        ng.ng_calibrate_many([])            # nothing to do
        calibrate_many([a, b])
        assert np.array_equal(_result(a)[0]["src"], _result(b)[0]["src"])
    finally:
        for n in (a, b, other):
            n.close()
