"""Pins of the oracle's autapse prohibition (allow_autapses = 0; the paper
names the flag as future work, Discussion), against definitions that do not
use it:

* ranges that do not overlap: identical to the call with autapses allowed;
* all_to_all: exactly the pairs (s, t), s != t, in row-major order (brute force);
* one_to_one: no connections when s0 == t0, else identical to the allowed call;
* fixed_total_number: every synapse whose first draw is not an autapse equals
  the allowed call's synapse (same words), and the pairs are uniform over the
  allowed pairs (chi-square);
* fixed_in/outdegree: exact degrees, never s == t, and the drawn nodes uniform
  over the range without the node itself (chi-square);
* calls that can only make autapses are rejected.
"""
from types import SimpleNamespace

import numpy as np
import pytest
from scipy import stats

import oracle


def _call(rule, src, tgt, k, allow=0, d=("uniform_int", 1, 9)):
    return SimpleNamespace(rule=rule, src=src, tgt=tgt, k_or_n=k, weight=("normal", 0.5, 0.05), delay=d,
                           allow_autapses=allow)


RULES = [("one_to_one", 0), ("all_to_all", 0), ("fixed_indegree", 9), ("fixed_outdegree", 8),
         ("fixed_total_number", 700)]


@pytest.mark.parametrize("rule,k", RULES)
def test_disjoint_ranges_unchanged(rule, k):
    src, tgt = (0, 30), (40, 30 if rule == "one_to_one" else 25)
    a = oracle.connect(3, 0.1, 2, _call(rule, src, tgt, k, allow=1))
    b = oracle.connect(3, 0.1, 2, _call(rule, src, tgt, k, allow=0))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("rule,k", RULES)
def test_no_self_connections(rule, k):
    src, tgt = (10, 30), (25, 30)  # nodes 25..39 in both
    s, t, _, _ = oracle.connect(5, 0.1, 1, _call(rule, src, tgt, k))
    assert s.size > 0 and not np.any(s == t)


def test_all_to_all_brute_force():
    src, tgt = (3, 7), (5, 6)
    s, t, _, _ = oracle.connect(1, 0.1, 0, _call("all_to_all", src, tgt, 0))
    want = [(a, b) for a in range(3, 10) for b in range(5, 11) if a != b]
    assert list(zip(s.tolist(), t.tolist())) == want
    # a target range of one node inside the source range: that source's row is empty
    s, t, _, _ = oracle.connect(1, 0.1, 0, _call("all_to_all", (0, 4), (2, 1), 0))
    assert list(zip(s.tolist(), t.tolist())) == [(0, 2), (1, 2), (3, 2)]


def test_one_to_one():
    assert oracle.count(_call("one_to_one", (4, 10), (4, 10), 0)) == 0
    a = oracle.connect(2, 0.1, 0, _call("one_to_one", (4, 10), (5, 10), 0, allow=1))
    b = oracle.connect(2, 0.1, 0, _call("one_to_one", (4, 10), (5, 10), 0, allow=0))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_fixed_total_number_shares_words_and_is_uniform():
    src = tgt = (0, 5)
    n = 40_000
    s1, t1, w1, d1 = oracle.connect(7, 0.1, 3, _call("fixed_total_number", src, tgt, n, allow=1))
    s0, t0, w0, d0 = oracle.connect(7, 0.1, 3, _call("fixed_total_number", src, tgt, n, allow=0))
    keep = s1 != t1
    assert keep.mean() > 0.7
    assert np.array_equal(s0[keep], s1[keep]) and np.array_equal(t0[keep], t1[keep])
    assert np.array_equal(w0, w1) and np.array_equal(d0, d1)  # weights and delays keep their words
    assert not np.any(s0 == t0)
    counts = np.bincount(s0.astype(np.int64) * 5 + t0, minlength=25).reshape(5, 5)
    off = counts[~np.eye(5, dtype=bool)]
    assert stats.chisquare(off).pvalue > 1e-3


@pytest.mark.parametrize("rule", ["fixed_indegree", "fixed_outdegree"])
def test_degree_rules_uniform_without_self(rule):
    k = 6000
    c = _call(rule, (0, 8), (3, 2), k) if rule == "fixed_indegree" else _call(rule, (3, 2), (0, 8), k)
    s, t, _, _ = oracle.connect(11, 0.1, 4, c)
    assert not np.any(s == t)
    fixed, drawn = (t, s) if rule == "fixed_indegree" else (s, t)
    for node in np.unique(fixed):
        sel = drawn[fixed == node]
        assert sel.size == k
        others = [x for x in range(8) if x != node]
        counts = np.array([(sel == x).sum() for x in others])
        assert counts.sum() == k and stats.chisquare(counts).pvalue > 1e-3


def test_impossible_calls_rejected():
    assert oracle.count(_call("fixed_indegree", (5, 1), (5, 3), 2)) == -1
    assert oracle.count(_call("fixed_outdegree", (5, 3), (6, 1), 2)) == -1
    assert oracle.count(_call("fixed_total_number", (5, 1), (5, 1), 3)) == -1
    assert oracle.count(_call("fixed_total_number", (5, 1), (5, 1), 0)) == 0
