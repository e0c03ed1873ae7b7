"""GPU parity of pairwise_bernoulli (the Discussion names it as missing;
counted on the device, allocated exactly, then written), through the C ABI,
against the CPU oracle: creation order and calibrated arrays element by
element; p = 0 and p = 1; rows longer than one 4,096-pair unit; self-pairs
prohibited; mixed with other rules; and the error paths."""
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

N_NODES = 12_000


def _pb(p, src, tgt, allow=1, w=("normal", 0.5, 0.05), d=("uniform_int", 1, 25)):
    c = SimpleNamespace(rule="pairwise_bernoulli", src=src, tgt=tgt, k_or_n=0, weight=w, delay=d,
                        allow_autapses=allow, p=p)
    return c


def _other(rule, src, tgt, k, w=("normal", -0.5, 0.05), d=("uniform", 0.1, 3.0)):
    return SimpleNamespace(rule=rule, src=src, tgt=tgt, k_or_n=k, weight=w, delay=d)


def _counts(calls, seed):
    return [oracle.count_pairwise(seed, cid, c) for cid, c in enumerate(calls)]


def _check(calls, seed=77):
    ns = _counts(calls, seed)
    for c, n in zip(calls, ns):
        c.n_syn = (lambda n: lambda: n)(n)
    ref = oracle.build_network(seed, 0.1, N_NODES, calls)
    with Network(seed, 0.1, 1 << 16, 512 << 20) as net:
        net.create(N_NODES)
        got_n = [net.connect(c)[2] for c in calls]
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    assert got_n == ns
    check_creation_order(created, ref, calls)
    check_calibrated(out, gp, gs, ref, calls)


CASES = {
    "p0": [_pb(0.0, (0, 100), (100, 100))],
    "p1_is_all_to_all": [_pb(1.0, (0, 40), (30, 70))],
    "long_rows": [_pb(0.05, (0, 30), (1000, 10_000))],  # 3 units per row, the last partial
    "no_autapses": [_pb(0.3, (0, 300), (200, 300), allow=0)],
    "ms_delays_uniform_weights": [_pb(0.2, (500, 200), (0, 5000), w=("uniform", -1.0, 1.0),
                                      d=("uniform", 0.05, 2.5))],
    "mixed": [_other("fixed_total_number", (0, 400), (400, 400), 30_000), _pb(0.1, (400, 400), (0, 700)),
              _other("fixed_indegree", (0, 100), (100, 50), 17)],
    # 21 connections first: the pairwise call starts at a position that is not a multiple of 4
    "unaligned_start": [_other("fixed_indegree", (0, 100), (100, 3), 7), _pb(0.15, (0, 300), (0, 2000))],
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_pairwise_matches_oracle(name):
    _check(CASES[name])


def test_pairwise_errors_change_nothing():
    with Network(1, 0.1, 1 << 16, 4 << 20) as net:  # an arena too small for 1e6 connections
        net.create(2000)
        for bad, status in [(_pb(1.5, (0, 10), (0, 10)), ng.NG_ERR_INVALID_ARG),
                            (_pb(0.5, (0, 10), (1995, 10)), ng.NG_ERR_INVALID_ARG),
                            (_pb(1.0, (0, 1000), (1000, 1000)), ng.NG_ERR_OOM)]:
            with pytest.raises(ng.NGError) as e:
                net.connect(bad)
            assert e.value.status == status
        assert net.view().n_conns == 0
        assert net.connect(_pb(0.5, (0, 10), (0, 10)))[0] == 0  # first call id still free
        with pytest.raises(ng.NGError) as e:
            net.connect_batch([_pb(0.5, (0, 10), (0, 10))])
        assert e.value.status == ng.NG_ERR_UNSUPPORTED


def test_pairwise_without_room_for_the_decisions():
    # 2,000 x 4,096 pairs: the counting pass keeps 1 MB of decisions; the
    # arena then has no room for the one block of connections, so the
    # decisions are dropped and the writing pass evaluates the pairs again
    call = _pb(0.0075, (0, 2000), (2000, 4096))
    n = oracle.count_pairwise(5, 0, call)
    assert 0 < n < (1 << 16)
    call.n_syn = lambda: n
    ref = oracle.build_network(5, 0.1, 6200, [call])
    with Network(5, 0.1, 1 << 16, 1_100_000) as net:
        net.create(6200)
        assert net.connect(call)[2] == n
        created = net.fetch()
    check_creation_order(created, ref, [call])


def test_pairwise_full_size_sampled():
    """The benchmark's call at full size (all 77,169 microcircuit nodes to the first 50,000,
    p = 0.0777: 3.86e9 pairs, ~3.0e8 connections, blocks of 2^24, the bench's sort schedule):
    sampled source rows against the oracle's row decisions, bit for bit, with their delays and
    weights by connection index; after calibration, each sampled source's run is its creation
    run stably sorted by delay and the group index marks the delay changes."""
    from paper_2306_09855_amd import workloads as W
    from paper_2306_09855_amd.network import arena_bytes_for
    from parity import check_equal, check_weights

    wl = W.microcircuit()
    n_tgt, p, B = 50_000, 0.0777, 1 << 24
    call = _pb(p, (0, wl.n_nodes), (0, n_tgt), w=("normal", 0.5, 0.05), d=("uniform_int", 1, 30))
    arena = arena_bytes_for(int(wl.n_nodes * n_tgt * p * 1.01), wl.n_nodes, wl.max_delay, B, 9) + (64 << 20)
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([[0, 1, 12_345, 49_999, 50_000, wl.n_nodes - 1],
                                     rng.integers(0, wl.n_nodes, 18)]))
    with Network(wl.seed, wl.h, B, arena) as net:
        net.tune(9, 1024)
        net.create(wl.n_nodes)
        cid, first, n = net.connect(call)
        assert first == 0 and abs(n - wl.n_nodes * n_tgt * p) < 6 * np.sqrt(wl.n_nodes * n_tgt * p)
        dev = net.fetch(device=True)
        lo = torch.searchsorted(dev["src"], torch.from_numpy(rows.astype(np.int32)).cuda()).cpu().numpy()
        hi = torch.searchsorted(dev["src"], torch.from_numpy(rows.astype(np.int32)).cuda(), right=True).cpu().numpy()
        created = {}
        for a, l, h in zip(rows, lo, hi):
            want = oracle.pairwise_row(wl.seed, cid, call, int(a))
            t = dev["tgt"][l:h].cpu().numpy()
            check_equal(t, want, f"targets of source {a}")
            w = dev["w"][l:h].cpu().numpy()
            d = dev["delay"][l:h].cpu().numpy()
            ref = [oracle.pairwise_values(wl.seed, wl.h, cid, call, int(j)) for j in range(l, h)]
            check_equal(d, [r[1] for r in ref], f"delays of source {a}")
            check_weights(w, np.array([r[0] for r in ref]), np.full(h - l, 0.5), f"weights of source {a}")
            created[int(a)] = (t, w, d)
        del dev
        net.calibrate()
        out = net.fetch(device=True)
        gp, gs = net.group_index()
        for a in rows:
            t, w, d = created[int(a)]
            l = int(torch.searchsorted(out["src"], torch.tensor([int(a)], dtype=torch.int32, device="cuda")).item())
            order = np.argsort(d, kind="stable")  # the run of a, stably sorted by delay
            check_equal(out["tgt"][l:l + t.size].cpu().numpy(), t[order], f"sorted targets of source {a}")
            check_equal(out["delay"][l:l + t.size].cpu().numpy(), d[order], f"sorted delays of source {a}")
            assert np.array_equal(out["w"][l:l + t.size].cpu().numpy(), w[order])
            starts = l + np.concatenate([[0], np.nonzero(np.diff(d[order]))[0] + 1]) if t.size else np.zeros(0)
            check_equal(gs[gp[a]:gp[a + 1]], starts, f"group starts of source {a}")
