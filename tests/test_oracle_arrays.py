"""Pins of the oracle's node arrays and per-connection weight/delay arrays
(Sec. 2.1, last paragraphs), by reduction to cases pinned elsewhere:

* an index array holding the consecutive range gives exactly the range call;
* any index array gives the range call taken from 0, mapped through the array
  (the formulas give array positions);
* a weight array leaves sources, targets and delays of the call unchanged
  (weights draw from their own stream) and its values come out exactly;
* a delay array consumes no delay word: sources and targets equal those of
  the call with a constant delay, and delays that are whole multiples of the
  step, or below one step, come out as those multiples, or as one step.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W

RULE_CASES = [
    ("one_to_one", 37, 37, 0),
    ("all_to_all", 13, 9, 0),
    ("fixed_indegree", 23, 17, 5),
    ("fixed_outdegree", 19, 29, 4),
    ("fixed_total_number", 31, 41, 500),
]


def _call(rule, ns, nt, k, s0=5, t0=100, w=("normal", 0.5, 0.05), d=("uniform_int", 1, 9), **arrays):
    c = SimpleNamespace(rule=rule, src=(s0, ns), tgt=(t0, nt), k_or_n=k, weight=w, delay=d)
    for name, a in arrays.items():
        setattr(c, name, a)
        if name == "src_idx":
            c.src = (0, len(a))
        if name == "tgt_idx":
            c.tgt = (0, len(a))
    return c


@pytest.mark.parametrize("rule,ns,nt,k", RULE_CASES)
def test_identity_arrays_equal_ranges(rule, ns, nt, k):
    base = oracle.connect(9, 0.1, 3, _call(rule, ns, nt, k))
    arr = oracle.connect(9, 0.1, 3, _call(rule, ns, nt, k, src_idx=np.arange(5, 5 + ns),
                                          tgt_idx=np.arange(100, 100 + nt)))
    for a, b in zip(base, arr):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("rule,ns,nt,k", RULE_CASES)
def test_arrays_map_positions(rule, ns, nt, k):
    rng = np.random.default_rng(ns * nt)
    sidx = rng.integers(0, 1000, ns).astype(np.uint32)  # repeats allowed
    tidx = rng.permutation(2000)[:nt].astype(np.uint32)
    pos = oracle.connect(4, 0.1, 2, _call(rule, ns, nt, k, s0=0, t0=0))
    got = oracle.connect(4, 0.1, 2, _call(rule, ns, nt, k, src_idx=sidx, tgt_idx=tidx))
    assert np.array_equal(got[0], sidx[pos[0]])
    assert np.array_equal(got[1], tidx[pos[1]])
    assert np.array_equal(got[2], pos[2]) and np.array_equal(got[3], pos[3])


@pytest.mark.parametrize("rule,ns,nt,k", RULE_CASES)
def test_weight_array(rule, ns, nt, k):
    c = _call(rule, ns, nt, k)
    n = oracle.count(c)
    wa = np.random.default_rng(1).normal(0, 3, n).astype(np.float32)
    base = oracle.connect(2, 0.1, 7, c)
    got = oracle.connect(2, 0.1, 7, _call(rule, ns, nt, k, w_arr=wa))
    assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])
    assert np.array_equal(got[3], base[3])
    assert np.array_equal(got[2], wa.astype(np.float64))


@pytest.mark.parametrize("rule,ns,nt,k", RULE_CASES)
def test_delay_array(rule, ns, nt, k):
    h = 0.125  # a power of two: d_ms = m * h is exact in fp32
    c_const = _call(rule, ns, nt, k, d=("const", 1.0))
    n = oracle.count(c_const)
    rng = np.random.default_rng(2)
    steps = rng.integers(1, 300, n)
    d_ms = (steps * h).astype(np.float32)
    small = rng.random(n) < 0.2  # below one step: one step
    d_ms[small] = np.float32(0.4 * h)
    steps[small] = 1
    base = oracle.connect(3, h, 1, c_const)
    got = oracle.connect(3, h, 1, _call(rule, ns, nt, k, d=("uniform_int", 1, 9), d_arr=d_ms))
    assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])
    assert np.array_equal(got[2], base[2])
    assert np.array_equal(got[3], steps)
    assert oracle.words_per_synapse(_call(rule, ns, nt, k, d_arr=d_ms)) == \
        oracle.words_per_synapse(c_const)
