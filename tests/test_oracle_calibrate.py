"""Pins of the oracle's calibration (Sec. 2.2, Eq. (14)).

The calibrated order is the plain definition "source first, delay second", and
the order of connections with equal keys is taken to be their creation order
(a stable sort).  The tests compare against Python's own stable ``sorted`` on
small inputs, and check the group index against brute-force sets.
"""
import numpy as np
import pytest

import oracle


def _random_input(rng, n, n_nodes, max_delay, src_hi=None):
    src = rng.integers(0, src_hi or n_nodes, n).astype(np.uint32)
    d = rng.integers(1, max_delay + 1, n).astype(np.int32)
    return src, d


@pytest.mark.parametrize("n,n_nodes,max_delay", [(0, 5, 3), (1, 1, 1), (17, 4, 3), (500, 40, 7),
                                                  (3000, 1000, 20), (2000, 3, 2)])
def test_sort_matches_python_stable_sort(n, n_nodes, max_delay):
    rng = np.random.default_rng(n + n_nodes)
    src, d = _random_input(rng, n, n_nodes, max_delay)
    perm, gptr, gstart = oracle.calibrate(n_nodes, src, d)
    expected = sorted(range(n), key=lambda j: (int(src[j]), int(d[j])))
    assert perm.tolist() == expected


def test_group_index_brute_force():
    rng = np.random.default_rng(1)
    n, n_nodes = 5000, 300
    src, d = _random_input(rng, n, n_nodes, 9, src_hi=250)   # nodes 250..299 have no outputs
    perm, gptr, gstart = oracle.calibrate(n_nodes, src, d)
    s_src, s_d = src[perm], d[perm]
    # G_i = number of distinct delays among the connections of source i
    G = np.array([len(set(d[src == i].tolist())) for i in range(n_nodes)])
    assert gptr.size == n_nodes + 1
    assert gptr[0] == 0
    assert np.array_equal(np.diff(gptr.astype(np.int64)), G)       # Eq. (14)
    assert gptr[-1] == G.sum() == gstart.size - 1
    assert gstart[0] == 0 and gstart[-1] == n
    # every group holds one (source, delay), adjacent groups differ
    for g in range(gstart.size - 1):
        a, b = gstart[g], gstart[g + 1]
        assert b > a
        assert np.all(s_src[a:b] == s_src[a]) and np.all(s_d[a:b] == s_d[a])
        if g:
            assert (s_src[a], s_d[a]) != (s_src[a - 1], s_d[a - 1])
    # the groups of source i are group_ptr[i] .. group_ptr[i+1]-1
    for i in (0, 1, 100, 249, 250, 299):
        for g in range(gptr[i], gptr[i + 1]):
            assert s_src[gstart[g]] == i


def test_stability_within_groups():
    rng = np.random.default_rng(7)
    src, d = _random_input(rng, 20000, 50, 3)
    perm, _, gstart = oracle.calibrate(50, src, d)
    for g in range(gstart.size - 1):
        seg = perm[gstart[g]:gstart[g + 1]].astype(np.int64)
        assert np.all(np.diff(seg) > 0)


def test_recalibration_matches_single_calibration():
    # connect(A); calibrate; connect(B); calibrate == connect(A); connect(B); calibrate
    rng = np.random.default_rng(3)
    sA, dA = _random_input(rng, 3000, 100, 5)
    sB, dB = _random_input(rng, 2000, 100, 5)
    pA, _, _ = oracle.calibrate(100, sA, dA)
    s1 = np.concatenate([sA[pA], sB]); d1 = np.concatenate([dA[pA], dB])
    p1, g1, st1 = oracle.calibrate(100, s1, d1)
    s2 = np.concatenate([sA, sB]); d2 = np.concatenate([dA, dB])
    p2, g2, st2 = oracle.calibrate(100, s2, d2)
    ids1 = np.concatenate([pA, np.arange(3000, 5000)])[p1]
    assert np.array_equal(ids1, p2)
    assert np.array_equal(g1, g2) and np.array_equal(st1, st2)


def test_source_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.calibrate(3, np.array([0, 3], np.uint32), np.array([1, 1], np.int32))


def test_network_end_to_end_small():
    from paper_2306_09855_amd.workloads import two_pop_indegree
    wl = two_pop_indegree(scale=0.1)
    net = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
    n = wl.n_syn
    assert net["s_src"].size == n
    key = net["s_src"].astype(np.int64) * 64 + net["s_delay"]
    assert np.all(np.diff(key) >= 0)
    # the multiset of connections is preserved by calibration
    a = sorted(zip(net["src"].tolist(), net["tgt"].tolist(), net["delay"].tolist(), net["w"].tolist()))
    b = sorted(zip(net["s_src"].tolist(), net["s_tgt"].tolist(), net["s_delay"].tolist(), net["s_w"].tolist()))
    assert a == b
