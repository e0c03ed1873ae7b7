"""Pins of the oracle's COPASS block sort (Appendix A) against definitions
that do not use it.

* The partition of sorted subarrays for a total m, with ties broken toward
  lower subarray indices, is unique: m_i is the number of elements of
  subarray i among the first m of the stable order of all elements ordered by
  (value, subarray, position).  That count is computed by brute force.
* Partition invariants of the appendix: sum m_i = m, every left element <=
  every right element.
* Both last steps of the partition (threshold found; all brackets of width
  one) are reached on the random cases.
* The block sort equals numpy's stable argsort of the whole array (values and
  the carried creation index), for ragged last blocks, one block, blocks of
  one element, and heavy ties.
"""
import numpy as np
import pytest

import oracle


def _brute(subs, m):
    triples = [(int(v), i, j) for i, a in enumerate(subs) for j, v in enumerate(a)]
    triples.sort()
    out = np.zeros(len(subs), np.int64)
    for _, i, _ in triples[:m]:
        out[i] += 1
    return out


def _random_subs(rng, k, max_len, vmax):
    return [np.sort(rng.integers(0, vmax, rng.integers(0, max_len + 1))).astype(np.uint64) for _ in range(k)]


@pytest.mark.parametrize("vmax", [2, 5, 50, 1 << 40])
def test_partition_matches_stable_prefix(vmax):
    rng = np.random.default_rng(vmax)
    paths = set()
    for _ in range(300):
        subs = _random_subs(rng, int(rng.integers(1, 9)), 12, vmax)
        total = sum(a.size for a in subs)
        if total == 0:
            continue
        m = int(rng.integers(0, total + 1))
        mi, path, _ = oracle.copass_partition(subs, m)
        assert np.array_equal(mi, _brute(subs, m)), (subs, m)
        assert int(mi.sum()) == m
        left = [a[:c] for a, c in zip(subs, mi) if c]
        right = [a[c:] for a, c in zip(subs, mi) if c < a.size]
        if left and right:
            assert max(int(x.max()) for x in left) <= min(int(x.min()) for x in right)
        paths.add(path)
    if vmax > 2:
        assert {1, 2} <= paths, paths


def test_partition_all_equal_and_single():
    subs = [np.full(7, 3, np.uint64), np.full(5, 3, np.uint64), np.full(0, 3, np.uint64)]
    for m in range(1, 12):
        mi, path, _ = oracle.copass_partition(subs, m)
        assert np.array_equal(mi, _brute(subs, m))
    # one subarray: the prefix itself
    a = np.sort(np.random.default_rng(1).integers(0, 100, 40)).astype(np.uint64)
    for m in (1, 17, 39):
        mi, _, _ = oracle.copass_partition([a], m)
        assert mi.tolist() == [m]


def test_partition_iterations_logarithmic():
    rng = np.random.default_rng(7)
    subs = [np.sort(rng.integers(0, 1 << 30, 4096)).astype(np.uint64) for _ in range(16)]
    _, _, iters = oracle.copass_partition(subs, 4096 * 5 + 123)
    assert iters <= 16 * 13  # each bisection halves the widest bracket


@pytest.mark.parametrize("n,B,vmax", [(1, 1, 3), (10, 1, 3), (100, 7, 4), (257, 32, 1000),
                                      (64, 64, 10), (63, 64, 10), (1000, 100, 2), (2048, 100, 1 << 22),
                                      (5000, 333, 30)])
def test_block_sort_equals_stable_sort(n, B, vmax):
    rng = np.random.default_rng(n * 31 + B)
    v = rng.integers(0, vmax, n).astype(np.uint64)
    out_v, out_p = oracle.copass_block_sort(v, B)
    order = np.argsort(v, kind="stable")
    assert np.array_equal(out_v, v[order])
    assert np.array_equal(out_p, order.astype(np.uint64))


def test_block_sort_single_block_is_the_underlying_sort():
    rng = np.random.default_rng(3)
    v = rng.integers(0, 9, 50).astype(np.uint64)
    out_v, out_p = oracle.copass_block_sort(v, 64)
    assert np.array_equal(out_p, np.argsort(v, kind="stable").astype(np.uint64))
