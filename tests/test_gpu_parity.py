"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle.

Sources, targets, delays and group offsets are compared bit for bit; weights
to the bound stated in tests/parity.py.  Sizes are chosen so the oracle
finishes in seconds while the GPU path still spans many sort tiles, several
ranges, several blocks (block size 2^16 in some cases) and ragged tails.
"""
import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W
from parity import check_calibrated, check_creation_order, check_equal, check_weights, per_record_base

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd import ng  # noqa: E402
from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402


def _net(wl, block_size=0, arena=None):
    return Network(wl.seed, wl.h, block_size,
                   arena or arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, block_size or (1 << 24)))


def _gpu_run(wl, block_size=0, batched=False, tuning=None, calibration="radix"):
    with _net(wl, block_size) as net:
        net.set_calibration(calibration)
        if tuning:
            net.tune(*tuning)
        net.build(wl, batched=batched, calibrate=False)
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    return created, out, gp, gs


def _check_all(wl, **kw):
    ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
    created, out, gp, gs = _gpu_run(wl, **kw)
    check_creation_order(created, ref, wl.calls)
    check_calibrated(out, gp, gs, ref, wl.calls)
    return ref, out


def _two_pop(rule, n=1500, k=7, w=("normal", 0.5, 0.05), d=("uniform_int", 1, 20), seed=12345, ntot=23_457):
    calls = [W.Call(rule, (0, n), (n, n) if rule != "one_to_one" else (n, n),
                    ntot if rule == "fixed_total_number" else k, w, d)]
    return W.Workload(f"two_pop_{rule}", seed, [n, n], calls)


@pytest.mark.parametrize("rule", W.RULES)
def test_each_rule_small_blocks(rule):
    # block size 2^16 so that calls straddle blocks
    wl = _two_pop(rule, n=300 if rule == "all_to_all" else 5000, k=13)
    _check_all(wl, block_size=1 << 16)


@pytest.mark.parametrize("w,d", [
    (("const", -1.25), ("const", 1.0)),
    (("uniform", -0.5, 2.0), ("uniform", 0.05, 3.0)),
    (("normal", 0.0, 1.0), ("uniform_int", 3, 3)),
    (("normal", -0.5, 0.05), ("uniform", 0.0, 0.3)),      # ms delays below one step clamp to 1
    (("const", 0.0), ("uniform_int", 1, 32767)),           # widest int16 delays: 15 delay bits
])
def test_weight_and_delay_kinds(w, d):
    wl = _two_pop("fixed_total_number", n=2000, w=w, d=d, ntot=40_001)
    _check_all(wl)


def test_two_pop_indegree_1e5():
    # two populations of 1,000 nodes, A->B fixed_indegree K=100: 1e5 synapses
    ref, out = _check_all(W.two_pop_indegree())
    assert out["src"].size == 100_000


def test_microcircuit_scaled():
    # the 64-call microcircuit shape at 1/20 of its node count: 750k synapses
    wl = W.microcircuit(scale=0.05)
    _check_all(wl, block_size=1 << 18)


def test_two_pop_mixed_scaled():
    wl = W.two_pop_mixed(scale=0.03)
    _check_all(wl)


def test_batch_equals_plain_and_oracle():
    wl = W.batch_mixed(n_calls=300, n_nodes=200_000, lo_exp=1.0, hi_exp=4.2, gen_seed=7)
    ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
    c1, o1, gp1, gs1 = _gpu_run(wl, batched=False)
    c2, o2, gp2, gs2 = _gpu_run(wl, batched=True)
    for k in ("src", "tgt", "delay", "w"):
        assert np.array_equal(c1[k], c2[k]) and np.array_equal(o1[k], o2[k]), k
    assert np.array_equal(gp1, gp2) and np.array_equal(gs1, gs2)
    check_creation_order(c2, ref, wl.calls)
    check_calibrated(o2, gp2, gs2, ref, wl.calls)


@pytest.mark.parametrize("tuning", [(4, 1024), (5, 1), (7, 3), (8, 9), (9, 100000)])
def test_schedule_invariance(tuning):
    # LSD form: digit widths 4..9 (2..5 passes) and range counts (a single
    # range, counts that are not multiples of 8, more ranges than tiles) give
    # identical results
    wl = W.microcircuit(scale=0.02)
    _check_all(wl, tuning=tuning, calibration="lsd")


def test_edge_cases():
    h = 0.1
    with Network(5, h, 1 << 16, 64 << 20) as net:
        # calibrate an empty context
        net.calibrate()
        gp, gs = net.group_index()
        assert gp.size == 1 and gs.tolist() == [0]
        a = net.create(1)
        # a single node, zero-sized calls, a one-synapse call
        cid, first, n = net.connect(W.Call("fixed_total_number", a, a, 0))
        assert n == 0
        cid, first, n = net.connect(W.Call("all_to_all", (0, 0), a))
        assert n == 0
        cid, first, n = net.connect(W.Call("fixed_total_number", a, a, 1, ("const", 2.0), ("const", 0.3)))
        assert (cid, first, n) == (2, 0, 1)
        net.calibrate()
        out = net.fetch()
        assert out["src"].tolist() == [0] and out["tgt"].tolist() == [0] and out["delay"].tolist() == [3]
        assert out["w"].tolist() == [2.0]
        gp, gs = net.group_index()
        assert gp.tolist() == [0, 1] and gs.tolist() == [0, 1]


@pytest.mark.parametrize("batched", [False, True])
def test_misaligned_calls(batched):
    # Calls of every size mod 4 leave every start position mod 4 in turn, so
    # generation stores aligned chunks assembled across lanes, across calls
    # (batched) and around wave and call edges; the calls cross several
    # 2^16-connection blocks.
    rng = np.random.default_rng(77)
    n = 3000
    calls = []
    for i in range(60):
        size = int(rng.integers(1, 9)) if i % 3 else int(rng.integers(3000, 9000))
        rule = ("fixed_total_number", "fixed_indegree", "one_to_one", "all_to_all", "fixed_outdegree")[i % 5]
        if rule == "fixed_total_number":
            calls.append(W.Call(rule, (0, n), (0, n), size))
        elif rule == "fixed_indegree":
            calls.append(W.Call(rule, (0, n), (int(rng.integers(0, n - 3)), 3), size))
        elif rule == "fixed_outdegree":
            calls.append(W.Call(rule, (int(rng.integers(0, n - 2)), 2), (0, n), size))
        elif rule == "one_to_one":
            k = min(size, n)
            calls.append(W.Call(rule, (0, k), (n - k, k)))
        else:
            calls.append(W.Call(rule, (0, min(size, n)), (0, 1 + i % 7)))
    wl = W.Workload("misaligned", 4321, [n], calls)
    _check_all(wl, block_size=1 << 16, batched=batched)


def test_connect_after_calibrate():
    # calibrate; connect more; calibrate == one calibration at the end
    wl = W.microcircuit(scale=0.02)
    half = len(wl.calls) // 2
    ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
    with _net(wl, 1 << 16) as net:
        for n in wl.populations:
            net.create(n)
        for c in wl.calls[:half]:
            net.connect(c)
        net.calibrate()
        net.calibrate()  # no-op
        for c in wl.calls[half:]:
            net.connect(c)
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    check_calibrated(out, gp, gs, ref, wl.calls)


def test_determinism():
    wl = W.microcircuit(scale=0.03)
    a = _gpu_run(wl)
    b = _gpu_run(wl, block_size=1 << 16)
    for x, y in zip(a[:2], b[:2]):
        for k in x:
            assert np.array_equal(x[k], y[k]), k
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_errors_leave_state_unchanged():
    wl = W.two_pop_indegree(scale=0.1)
    with Network(wl.seed, wl.h, 1 << 16, 8 << 20) as net:
        net.create(100)
        net.create(100)
        with pytest.raises(ng.NGError) as e:
            net.connect(W.Call("one_to_one", (0, 100), (100, 99)))
        assert e.value.status == ng.NG_ERR_INVALID_ARG
        with pytest.raises(ng.NGError) as e:      # does not fit the 8 MiB arena
            net.connect(W.Call("fixed_total_number", (0, 100), (100, 100), 2_000_000))
        assert e.value.status == ng.NG_ERR_OOM
        # the failed calls consumed no call id: this call is connect id 0
        cid, first, n = net.connect(wl.calls[0])
        assert (cid, first) == (0, 0)
        net.calibrate()
        out = net.fetch()
    ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
    check_equal(out["src"], ref["s_src"], "src")
    check_equal(out["tgt"], ref["s_tgt"], "tgt")


def test_set_seed():
    # a context reset and reseeded builds the network of the new seed; the
    # seed cannot change once a Connect call was issued
    wl = W.two_pop_indegree(scale=0.3)
    with _net(wl) as net:
        net.build(wl)
        with pytest.raises(ng.NGError) as e:
            ng.ng_set_seed(net.ctx, 99)
        assert e.value.status == ng.NG_ERR_STATE
        ng.ng_reset(net.ctx)
        ng.ng_set_seed(net.ctx, 99)
        net.build(wl)
        out = net.fetch()
        gp, gs = net.group_index()
    ref = oracle.build_network(99, wl.h, wl.n_nodes, wl.calls)
    check_calibrated(out, gp, gs, ref, wl.calls)
