"""Full-size parity: the microcircuit-shaped network of 77,169 nodes and
3.0e8 synapses in 64 fixed_total_number calls, in the launch configuration
the benchmark times (one ng_connect per call, then ng_calibrate).

The oracle cannot rebuild 3e8 synapses in test time, so:
  * creation order is checked element by element at sampled positions (every
    call's first and last synapse plus random ones), each recomputed by the
    oracle one synapse at a time;
  * the calibrated order is checked by properties that hold at any size:
    keys non-decreasing, and the result equals a stable sort (torch's, an
    independent implementation) of the checked creation-order arrays;
  * the group index is recomputed from the sorted keys with plain tensor ops.
"""
import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W
from parity import check_equal, check_weights

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402


@pytest.fixture(scope="module")
def microcircuit_full():
    wl = W.microcircuit()
    assert wl.n_syn == 300_000_000
    net = Network(wl.seed, wl.h, 0, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay))
    net.build(wl, calibrate=False)
    created = net.fetch(device=True)
    net.calibrate()
    out = net.fetch(device=True)
    gp, gs = net.group_index()
    net.close()
    yield wl, created, out, gp, gs
    del created, out
    torch.cuda.empty_cache()


def test_creation_order_sampled(microcircuit_full):
    wl, created, _, _, _ = microcircuit_full
    rng = np.random.default_rng(2024)
    starts = np.concatenate([[0], np.cumsum([c.n_syn() for c in wl.calls])])
    picks = [(c, 0) for c in range(len(wl.calls))] + [(c, wl.calls[c].n_syn() - 1) for c in range(len(wl.calls))]
    for pos in rng.integers(0, wl.n_syn, 3000):
        c = int(np.searchsorted(starts, pos, side="right") - 1)
        picks.append((c, int(pos - starts[c])))
    pos = np.array([starts[c] + i for c, i in picks], dtype=np.int64)
    ref = np.array([oracle.synapse(wl.seed, wl.h, c, wl.calls[c], i) for c, i in picks], dtype=object)
    idx = torch.from_numpy(pos).cuda()
    check_equal(created["src"][idx].cpu().numpy().view(np.uint32), ref[:, 0].astype(np.int64), "src")
    check_equal(created["tgt"][idx].cpu().numpy().view(np.uint32), ref[:, 1].astype(np.int64), "tgt")
    check_equal(created["delay"][idx].cpu().numpy(), ref[:, 3].astype(np.int64), "delay")
    base = np.array([wl.calls[c].weight[1] for c, _ in picks])
    check_weights(created["w"][idx].cpu().numpy(), ref[:, 2].astype(np.float64), base, "w")


def test_calibrated_is_stable_sort(microcircuit_full):
    wl, created, out, _, _ = microcircuit_full
    dbits = int(wl.max_delay).bit_length()
    key_c = (created["src"].to(torch.int64) << dbits) | created["delay"].to(torch.int64)
    key_s = (out["src"].to(torch.int64) << dbits) | out["delay"].to(torch.int64)
    assert bool((key_s[1:] >= key_s[:-1]).all())
    _, order = torch.sort(key_c, stable=True)
    del key_c
    for k in ("src", "tgt", "delay"):
        assert torch.equal(created[k][order], out[k]), k
    assert torch.equal(created["w"][order].view(torch.int32), out["w"].view(torch.int32))


def test_group_index_full(microcircuit_full):
    wl, _, out, gp, gs = microcircuit_full
    dbits = int(wl.max_delay).bit_length()
    key = (out["src"].to(torch.int64) << dbits) | out["delay"].to(torch.int64)
    flag = torch.ones_like(key, dtype=torch.bool)
    flag[1:] = key[1:] != key[:-1]
    starts = torch.nonzero(flag).flatten()
    G = int(starts.numel())
    assert gs.size == G + 1 and gs[-1] == wl.n_syn
    assert torch.equal(torch.from_numpy(gs[:-1].astype(np.int64)).cuda(), starts)
    per_src = torch.bincount(out["src"][starts].to(torch.int64), minlength=wl.n_nodes)
    ptr = torch.zeros(wl.n_nodes + 1, dtype=torch.int64, device="cuda")
    ptr[1:] = torch.cumsum(per_src, 0)
    assert torch.equal(torch.from_numpy(gp.astype(np.int64)).cuda(), ptr)


def test_many_output_blocks_stable_sort():
    # 4e7 synapses in blocks of 2^16 records: 611 output blocks, more than the
    # last sort pass keeps in LDS, so it reads the device block table instead
    wl = W.microcircuit(total=40_000_000)
    B = 1 << 16
    assert -(-wl.n_syn // B) > 512
    with Network(wl.seed, wl.h, B, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B)) as net:
        net.build(wl, calibrate=False)
        created = net.fetch(device=True)
        net.calibrate()
        out = net.fetch(device=True)
    dbits = int(wl.max_delay).bit_length()
    key_c = (created["src"].to(torch.int64) << dbits) | created["delay"].to(torch.int64)
    _, order = torch.sort(key_c, stable=True)
    for k in ("src", "tgt", "delay"):
        assert torch.equal(created[k][order], out[k]), k
    assert torch.equal(created["w"][order].view(torch.int32), out["w"].view(torch.int32))


def test_full_size_copass_equals_radix(microcircuit_full):
    # the COPASS in-place block sort (18 blocks of 2^24) gives the radix
    # path's arrays and group index bit for bit
    wl, _, out, gp, gs = microcircuit_full
    net = Network(wl.seed, wl.h, 0, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay))
    try:
        net.set_calibration("copass")
        net.build(wl)
        cp = net.fetch(device=True)
        gp2, gs2 = net.group_index()
    finally:
        net.close()
    for k in ("src", "tgt", "delay"):
        assert torch.equal(cp[k], out[k]), k
    assert torch.equal(cp["w"].view(torch.int32), out["w"].view(torch.int32))
    assert np.array_equal(gp2, gp) and np.array_equal(gs2, gs)


def test_no_autapses_no_multapses_full_size():
    """The microcircuit with allow_autapses = 0 and allow_multapses = 0 on all 64 calls, at
    full size in the benchmark's configuration (blocks of 2^24, 9-bit widest digit, 1,024
    ranges): sampled synapses of every call recomputed by the oracle one at a time; every
    call's pairs distinct and none a self-pair; the calibrated arrays a stable sort of the
    created ones."""
    from types import SimpleNamespace

    wl = W.microcircuit()
    calls = []
    for c in wl.calls:
        nc = SimpleNamespace(rule=c.rule, src=c.src, tgt=c.tgt, k_or_n=c.k_or_n, weight=c.weight, delay=c.delay,
                             allow_autapses=0, allow_multapses=0)
        nc.n_syn = (lambda x: (lambda: oracle.count(x)))(nc)
        calls.append(nc)
    B = 1 << 24
    net = Network(wl.seed, wl.h, B, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B, 9))
    try:
        net.tune(9, 1024)
        for n in wl.populations:
            net.create(n)
        firsts = [net.connect(c)[1] for c in calls]
        created = net.fetch(device=True)
        rng = np.random.default_rng(11)
        picks = []
        for ci, c in enumerate(calls):
            n = c.n_syn()
            picks += [(ci, 0), (ci, n - 1)] + [(ci, int(i)) for i in rng.integers(0, n, 40)]
        pos = np.array([firsts[ci] + i for ci, i in picks], dtype=np.int64)
        ref = np.array([oracle.synapse(wl.seed, wl.h, ci, calls[ci], i) for ci, i in picks], dtype=object)
        idx = torch.from_numpy(pos).cuda()
        check_equal(created["src"][idx].cpu().numpy().view(np.uint32), ref[:, 0].astype(np.int64), "src")
        check_equal(created["tgt"][idx].cpu().numpy().view(np.uint32), ref[:, 1].astype(np.int64), "tgt")
        check_equal(created["delay"][idx].cpu().numpy(), ref[:, 3].astype(np.int64), "delay")
        base = np.array([calls[ci].weight[1] for ci, _ in picks])
        check_weights(created["w"][idx].cpu().numpy(), ref[:, 2].astype(np.float64), base, "w")
        src = created["src"].to(torch.int64)
        tgt = created["tgt"].to(torch.int64)
        assert bool((src != tgt).all())
        for ci, c in enumerate(calls):
            a, b = firsts[ci], firsts[ci] + c.n_syn()
            pairs = src[a:b] * wl.n_nodes + tgt[a:b]
            assert torch.unique(pairs).numel() == b - a, f"call {ci}: a repeated pair"
        key = src * 65536 + created["delay"].to(torch.int64)  # delays are below 2^15
        order = torch.sort(key, stable=True).indices
        net.calibrate()
        out = net.fetch(device=True)
        for name in ("src", "tgt", "w", "delay"):
            assert torch.equal(out[name], created[name][order]), f"sorted {name}"
    finally:
        net.close()
        torch.cuda.empty_cache()


def test_node_and_value_arrays_full_size():
    """The benchmark's arrays build at full size: every call's source group an index array (a
    random permutation of its population), weights and delays (ms) per connection from device
    arrays, blocks of 2^24; sampled synapses of every call recomputed by the oracle with the
    same arrays; the calibrated arrays a stable sort of the created ones."""
    from types import SimpleNamespace

    wl = W.microcircuit()
    rng = np.random.default_rng(5)
    B = 1 << 24
    net = Network(wl.seed, wl.h, B, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B, 9))
    try:
        net.tune(9, 1024)
        for n in wl.populations:
            net.create(n)
        calls, firsts, keep = [], [], []
        for c in wl.calls:
            s0, ns = c.src
            nc = SimpleNamespace(rule=c.rule, src=(0, ns), tgt=c.tgt, k_or_n=c.k_or_n, weight=c.weight,
                                 delay=c.delay)
            n = oracle.count(nc)
            nc.src_idx = (s0 + rng.permutation(ns)).astype(np.uint32)
            nc.w_arr = rng.normal(0.5, 0.05, n).astype(np.float32)
            nc.d_arr = (rng.random(n) * 3.0).astype(np.float32)  # 1..30 steps at h = 0.1 ms
            dev = [torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).cuda()
                   for a in (nc.src_idx, nc.w_arr, nc.d_arr)]
            keep.append(dev)  # valid until the generation has run
            firsts.append(net.connect_groups(nc, dev[0], c.tgt, dev[1], dev[2])[1])
            calls.append(nc)
        torch.cuda.synchronize()
        created = net.fetch(device=True)
        picks = []
        for ci, c in enumerate(calls):
            n = c.w_arr.size
            picks += [(ci, 0), (ci, n - 1)] + [(ci, int(i)) for i in rng.integers(0, n, 40)]
        pos = np.array([firsts[ci] + i for ci, i in picks], dtype=np.int64)
        ref = np.array([oracle.synapse(wl.seed, wl.h, ci, calls[ci], i) for ci, i in picks], dtype=object)
        idx = torch.from_numpy(pos).cuda()
        check_equal(created["src"][idx].cpu().numpy().view(np.uint32), ref[:, 0].astype(np.int64), "src")
        check_equal(created["tgt"][idx].cpu().numpy().view(np.uint32), ref[:, 1].astype(np.int64), "tgt")
        check_equal(created["delay"][idx].cpu().numpy(), ref[:, 3].astype(np.int64), "delay")
        assert np.array_equal(created["w"][idx].cpu().numpy().astype(np.float64), ref[:, 2].astype(np.float64))
        key = created["src"].to(torch.int64) * 65536 + created["delay"].to(torch.int64)  # delays below 2^15
        order = torch.sort(key, stable=True).indices
        net.calibrate()
        out = net.fetch(device=True)
        for name in ("src", "tgt", "w", "delay"):
            assert torch.equal(out[name], created[name][order]), f"sorted {name}"
    finally:
        net.close()
        torch.cuda.empty_cache()
