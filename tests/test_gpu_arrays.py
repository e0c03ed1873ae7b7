"""GPU parity of node groups given as index arrays and of per-connection
weight and delay arrays (Sec. 2.1, last paragraphs), through the C ABI
(ng_connect_groups), against the CPU oracle: creation order and calibrated
arrays element by element, for every rule, mixed with range calls, and the
error paths (nothing changes, no call id is consumed)."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from parity import check_calibrated, check_creation_order

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd import ng  # noqa: E402
from paper_2306_09855_amd.network import Network  # noqa: E402

H = 0.1
N_NODES = 3000
RULES = [("one_to_one", 700, 700, 0), ("all_to_all", 90, 80, 0), ("fixed_indegree", 400, 300, 37),
         ("fixed_outdegree", 350, 500, 41), ("fixed_total_number", 600, 900, 70_001)]


def _call(rule, k, src, tgt, w=("normal", 0.5, 0.05), d=("uniform_int", 1, 40), **arrays):
    c = SimpleNamespace(rule=rule, k_or_n=k, weight=w, delay=d, src=src, tgt=tgt)
    for name, a in arrays.items():
        setattr(c, name, a)
    c.n_syn = lambda: oracle.count(c)
    return c


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda() if a is not None else None


def _run(seed, calls, block_size=1 << 16):
    """calls: list of (oracle call, gpu kwargs); returns created, calibrated, index."""
    with Network(seed, H, block_size, 256 << 20) as net:
        net.create(N_NODES)
        keep = []
        for c, kw in calls:
            src = kw.get("src_t", c.src)
            tgt = kw.get("tgt_t", c.tgt)
            keep += [kw.get("w_t"), kw.get("d_t"), src, tgt]
            net.connect_groups(c, src, tgt, kw.get("w_t"), kw.get("d_t"))
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    return created, out, gp, gs


def _check(seed, calls):
    ref = oracle.build_network(seed, H, N_NODES, [c for c, _ in calls])
    created, out, gp, gs = _run(seed, calls)
    check_creation_order(created, ref, [c for c, _ in calls])
    check_calibrated(out, gp, gs, ref, [c for c, _ in calls])


@pytest.mark.parametrize("which", ["src", "tgt", "both"])
@pytest.mark.parametrize("rule,ns,nt,k", RULES)
def test_index_arrays(rule, ns, nt, k, which):
    rng = np.random.default_rng(ns + nt + len(which))
    sidx = rng.integers(0, N_NODES, ns).astype(np.uint32) if which in ("src", "both") else None
    tidx = rng.permutation(N_NODES)[:nt].astype(np.uint32) if which in ("tgt", "both") else None
    kw, arrays = {}, {}
    src, tgt = (11, ns), (1500, nt)
    if sidx is not None:
        src, arrays["src_idx"], kw["src_t"] = (0, ns), sidx, _dev(sidx, torch.int32)
    if tidx is not None:
        tgt, arrays["tgt_idx"], kw["tgt_t"] = (0, nt), tidx, _dev(tidx, torch.int32)
    _check(17, [(_call(rule, k, src, tgt, **arrays), kw)])


@pytest.mark.parametrize("rule,ns,nt,k", RULES)
def test_weight_and_delay_arrays(rule, ns, nt, k):
    base = _call(rule, k, (0, ns), (ns, nt))
    n = oracle.count(base)
    rng = np.random.default_rng(n)
    w = rng.normal(0.0, 2.0, n).astype(np.float32)
    d = (rng.random(n) * 600.0).astype(np.float32)  # 0..600 ms: one step minimum, up to 6000 steps
    d[: n // 10] = np.float32(0.01)
    c = _call(rule, k, (0, ns), (ns, nt), w_arr=w, d_arr=d)
    _check(5, [(c, {"w_t": _dev(w, torch.float32), "d_t": _dev(d, torch.float32)})])


def test_value_arrays_not_16_byte_aligned():
    # views one element into a larger tensor: the per-connection values are read one by one
    base = _call("fixed_indegree", 23, (0, 300), (300, 200))
    n = oracle.count(base)
    rng = np.random.default_rng(3)
    w = rng.normal(0.0, 1.0, n).astype(np.float32)
    d = (rng.random(n) * 4.0).astype(np.float32)
    w_big = _dev(np.concatenate([[7.0], w]).astype(np.float32), torch.float32)
    d_big = _dev(np.concatenate([[7.0], d]).astype(np.float32), torch.float32)
    w_t, d_t = w_big[1:], d_big[1:]
    assert w_t.data_ptr() % 16 != 0 and d_t.data_ptr() % 16 != 0
    c = _call("fixed_indegree", 23, (0, 300), (300, 200), w_arr=w, d_arr=d)
    _check(8, [(c, {"w_t": w_t, "d_t": d_t})])


def test_array_calls_among_range_calls():
    rng = np.random.default_rng(9)
    sidx = rng.integers(0, N_NODES, 250).astype(np.uint32)
    w = rng.normal(1.0, 0.1, 250 * 12).astype(np.float32)
    calls = [
        (_call("fixed_total_number", 40_000, (0, 1000), (1000, 2000)), {}),
        (_call("fixed_outdegree", 12, (0, 250), (2000, 1000), src_idx=sidx, w_arr=w),
         {"src_t": _dev(sidx, torch.int32), "w_t": _dev(w, torch.float32)}),
        (_call("all_to_all", 0, (2500, 30), (0, 60), d=("uniform", 0.05, 3.0)), {}),
    ]
    _check(23, calls)


def test_array_errors_change_nothing():
    with Network(3, H, 1 << 16, 64 << 20) as net:
        net.create(100)
        good = _call("fixed_total_number", 500, (0, 100), (0, 100))
        bad_idx = _dev(np.array([3, 100, 7], np.uint32), torch.int32)  # 100 is not a node
        nan_d = _dev(np.array([1.0, np.nan] + [1.0] * 498, np.float32), torch.float32)
        big_d = _dev(np.full(500, 1e6, np.float32), torch.float32)  # 1e7 steps
        cases = [
            lambda: net.connect_groups(_call("all_to_all", 0, (0, 3), (0, 5)), bad_idx, (0, 5)),
            lambda: net.connect_groups(good, (0, 100), (0, 100), None, nan_d),
            lambda: net.connect_groups(good, (0, 100), (0, 100), None, big_d),
            lambda: net.connect_groups(_call("all_to_all", 0, (0, 3), (0, 5)),
                                       ng.ng_group(1, 3, bad_idx.data_ptr()), (0, 5)),
        ]
        for f in cases:
            with pytest.raises(ng.NGError) as e:
                f()
            assert e.value.status == ng.NG_ERR_INVALID_ARG
        assert net.view().n_conns == 0
        cid, first, n = net.connect_groups(good, (0, 100), (0, 100))
        assert (cid, first, n) == (0, 0, 500)
        spec = ng.conn_spec("all_to_all", 0)
        spec.allow_autapses = 0
        ok_idx = _dev(np.array([1, 2, 3], np.uint32), torch.int32)
        with pytest.raises(ng.NGError) as e:
            ng.ng_connect_groups(net.ctx, ng.group(ok_idx), ng.group((0, 5)), spec,
                                 ng.syn_spec(("const", 1.0), ("const", 1.0)))
        assert e.value.status == ng.NG_ERR_UNSUPPORTED
