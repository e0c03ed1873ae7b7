"""Pins of the oracle's multapse prohibition (allow_multapses = 0; future work
in the Discussion), defined with a keyed Feistel permutation walked into
[0, M):

* K = N_s (fixed_indegree) gives every target each source exactly once, and
  K = N_s - 1 without autapses each source but itself: the permutation is a
  bijection for every size tried; fixed_outdegree likewise;
* fixed_total_number with N = all pairs gives every pair exactly once (with
  and without self-pairs);
* with K < N_s the sources of a target are distinct and, over many targets,
  uniform (chi-square);
* delays: synapse i's delay is word i of the delay stream, the same as an
  all_to_all call's synapse i with the same call id;
* calls asking for more distinct draws than candidates are rejected.
"""
from types import SimpleNamespace

import numpy as np
import pytest
from scipy import stats

import oracle


def _call(rule, src, tgt, k, autapses=1, d=("uniform_int", 1, 20)):
    return SimpleNamespace(rule=rule, src=src, tgt=tgt, k_or_n=k, weight=("normal", 0.5, 0.05), delay=d,
                           allow_autapses=autapses, allow_multapses=0)


@pytest.mark.parametrize("ns", [1, 2, 3, 5, 17, 64, 100, 257])
def test_indegree_full_is_a_permutation(ns):
    s, t, _, _ = oracle.connect(3, 0.1, 1, _call("fixed_indegree", (0, ns), (1000, 7), ns))
    for tt in range(1000, 1007):
        assert sorted(s[t == tt].tolist()) == list(range(ns))


@pytest.mark.parametrize("n", [2, 3, 8, 33])
def test_full_without_autapses(n):
    s, t, _, _ = oracle.connect(5, 0.1, 2, _call("fixed_indegree", (0, n), (0, n), n - 1, autapses=0))
    for tt in range(n):
        assert sorted(s[t == tt].tolist()) == [x for x in range(n) if x != tt]
    s, t, _, _ = oracle.connect(5, 0.1, 2, _call("fixed_outdegree", (0, n), (0, n), n - 1, autapses=0))
    for ss in range(n):
        assert sorted(t[s == ss].tolist()) == [x for x in range(n) if x != ss]


@pytest.mark.parametrize("autapses", [1, 0])
def test_total_number_all_pairs_once(autapses):
    src, tgt = (0, 9), (4, 11)
    n = oracle.count(SimpleNamespace(rule="all_to_all", src=src, tgt=tgt, k_or_n=0, weight=("const", 1.0),
                                     delay=("const", 1.0), allow_autapses=autapses))
    s, t, _, _ = oracle.connect(8, 0.1, 0, _call("fixed_total_number", src, tgt, n, autapses=autapses))
    pairs = sorted(zip(s.tolist(), t.tolist()))
    want = sorted((a, b) for a in range(0, 9) for b in range(4, 15) if autapses or a != b)
    assert pairs == want


def test_distinct_and_uniform():
    k, ns = 40, 100
    s, t, _, _ = oracle.connect(11, 0.1, 4, _call("fixed_indegree", (0, ns), (0, 500), k))
    for tt in range(0, 500, 37):
        assert np.unique(s[t == tt]).size == k
    assert stats.chisquare(np.bincount(s, minlength=ns)).pvalue > 1e-3


def test_delay_words_match_all_to_all():
    c = _call("fixed_outdegree", (0, 30), (0, 50), 20)
    a2a = SimpleNamespace(rule="all_to_all", src=(0, 30), tgt=(0, 50), k_or_n=0, weight=("normal", 0.5, 0.05),
                          delay=("uniform_int", 1, 20))
    _, _, w, d = oracle.connect(6, 0.1, 9, c)
    _, _, wa, da = oracle.connect(6, 0.1, 9, a2a)
    assert np.array_equal(d, da[: d.size]) and np.array_equal(w, wa[: w.size])


def test_too_many_distinct_draws_rejected():
    assert oracle.count(_call("fixed_indegree", (0, 5), (10, 3), 6)) == -1
    assert oracle.count(_call("fixed_indegree", (0, 5), (0, 5), 5, autapses=0)) == -1
    assert oracle.count(_call("fixed_outdegree", (0, 3), (10, 4), 5)) == -1
    assert oracle.count(_call("fixed_total_number", (0, 3), (10, 4), 13)) == -1
    assert oracle.count(_call("fixed_total_number", (0, 3), (10, 4), 12)) == 12
