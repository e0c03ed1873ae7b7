"""Pins of the oracle's pairwise_bernoulli rule (named as missing in the
Discussion; defined here with per-pair decisions from the word streams):

* p = 0: no connections; p = 1: exactly all_to_all's pairs, in its order
  (and all_to_all's without autapses when they are prohibited);
* the number of connections is binomial(N_s N_t, p) (z test over seeds);
* targets and delays uniform (chi-square);
* connection j has the weight of synapse j of an all_to_all call with the
  same call id and weight law (weights are stream 1 of synapse j);
* the oracle's one-synapse path agrees with its whole-call path.
"""
from types import SimpleNamespace

import numpy as np
import pytest
from scipy import stats

import oracle


def _call(p, src=(0, 40), tgt=(30, 50), allow=1, w=("normal", 0.5, 0.1), d=("uniform_int", 1, 12)):
    return SimpleNamespace(rule="pairwise_bernoulli", src=src, tgt=tgt, k_or_n=0, weight=w, delay=d,
                           allow_autapses=allow, p=p)


def _a2a(src, tgt, allow=1, w=("normal", 0.5, 0.1), d=("uniform_int", 1, 12)):
    return SimpleNamespace(rule="all_to_all", src=src, tgt=tgt, k_or_n=0, weight=w, delay=d, allow_autapses=allow)


@pytest.mark.parametrize("allow", [1, 0])
def test_p_zero_and_one(allow):
    assert oracle.count_pairwise(3, 1, _call(0.0, allow=allow)) == 0
    s, t, w, _ = oracle.connect(3, 0.1, 1, _call(1.0, allow=allow))
    s2, t2, w2, _ = oracle.connect(3, 0.1, 1, _a2a((0, 40), (30, 50), allow=allow))
    assert np.array_equal(s, s2) and np.array_equal(t, t2)
    assert np.array_equal(w, w2)  # same weight words by connection index


def test_count_binomial():
    p, npairs = 0.1, 40 * 50
    counts = np.array([oracle.count_pairwise(seed, 0, _call(p)) for seed in range(200)])
    z = (counts.mean() - p * npairs) / np.sqrt(npairs * p * (1 - p) / len(counts))
    assert abs(z) < 4
    assert abs(counts.var() / (npairs * p * (1 - p)) - 1) < 0.35


def test_targets_and_delays_uniform():
    s, t, _, d = oracle.connect(9, 0.1, 2, _call(0.3, src=(0, 200), tgt=(0, 60), d=("uniform_int", 1, 10)))
    assert stats.chisquare(np.bincount(t, minlength=60)).pvalue > 1e-3
    assert stats.chisquare(np.bincount(d - 1, minlength=10)).pvalue > 1e-3
    assert np.all(np.diff(s.astype(np.int64) * 60 + t) > 0)  # pairs in row order, each once


def test_weights_share_the_connection_index():
    c = _call(0.25, w=("uniform", -1.0, 2.0))
    _, _, w, _ = oracle.connect(5, 0.1, 7, c)
    _, _, wa, _ = oracle.connect(5, 0.1, 7, _a2a((0, 40), (30, 50), w=("uniform", -1.0, 2.0)))
    assert np.array_equal(w, wa[: w.size])


def test_one_synapse_path_agrees():
    c = _call(0.2, allow=0, src=(0, 12), tgt=(5, 9), d=("uniform", 0.1, 2.0))
    s, t, w, d = oracle.connect(4, 0.1, 3, c)
    for i in range(0, s.size, 7):
        assert oracle.synapse(4, 0.1, 3, c, i) == (int(s[i]), int(t[i]), float(w[i]), int(d[i]))


@pytest.mark.parametrize("allow", [1, 0])
def test_row_and_value_paths_agree(allow):
    # the sampled-check helpers against the whole-call walk, and p = 1 / p = 0 rows in closed form
    c = _call(0.15, allow=allow, src=(0, 60), tgt=(20, 70), d=("uniform", 0.1, 2.0))
    s, t, w, d = oracle.connect(6, 0.1, 2, c)
    for a in range(60):
        run = np.nonzero(s == a)[0]
        assert np.array_equal(oracle.pairwise_row(6, 2, c, a), (t[run] - 20).astype(np.uint32))
    for j in range(0, s.size, 5):
        assert oracle.pairwise_values(6, 0.1, 2, c, j) == (float(w[j]), int(d[j]))
    full = oracle.pairwise_row(6, 2, _call(1.0, allow=allow, src=(0, 60), tgt=(20, 70)), 25)
    want = np.arange(70, dtype=np.uint32)
    if not allow:
        want = want[want != 25 - 20]  # source 25 is target offset 5
    assert np.array_equal(full, want)
    assert oracle.pairwise_row(6, 2, _call(0.0, allow=allow, src=(0, 60), tgt=(20, 70)), 25).size == 0
