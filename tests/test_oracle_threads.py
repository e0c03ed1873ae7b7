"""The oracle's timed mode (OpenMP over synapse indices, a sample sort for
calibration) against its single-thread reference mode: the same bytes.

Each synapse is a function of (seed, call, index) alone, and the calibration
order -- source, then delay (Sec. 2.2), ties by creation index -- is total, so
any thread count must give identical arrays.  The cases cover every rule, the
autapse and multapse prohibitions, node and value arrays, and sizes above the
sample sort's threshold (65,536 records), including heavy key ties.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle

H = 0.1


def _c(rule, src, tgt, k, **kw):
    d = dict(weight=("normal", 0.5, 0.05), delay=("uniform_int", 1, 20))
    d.update(kw)
    return SimpleNamespace(rule=rule, src=src, tgt=tgt, k_or_n=k, **d)


CASES = {
    "mixed": (3000, [
        _c("fixed_indegree", (0, 1000), (1000, 2000), 60),
        _c("fixed_outdegree", (1000, 1000), (0, 3000), 40),
        _c("fixed_total_number", (0, 3000), (0, 3000), 90_000, allow_autapses=0),
        _c("all_to_all", (2000, 300), (2100, 250), 0, allow_autapses=0),
        _c("one_to_one", (0, 1500), (1500, 1500), 0, delay=("uniform", 0.1, 3.0)),
    ]),
    "no_multapses": (2000, [
        _c("fixed_indegree", (0, 2000), (0, 2000), 50, allow_multapses=0, allow_autapses=0),
        _c("fixed_total_number", (0, 500), (500, 400), 150_000, allow_multapses=0),
    ]),
    "ties": (4, [  # four sources, one delay: keys shared by ~10^5 records each
        _c("fixed_total_number", (0, 4), (0, 4), 400_000, delay=("const", 0.1)),
    ]),
}


def _build(n_nodes, calls, seed, threads):
    with oracle.threads(threads):
        return oracle.build_network(seed, H, n_nodes, calls)


@pytest.mark.parametrize("case", sorted(CASES))
def test_threads_give_the_same_bytes(case):
    n_nodes, calls = CASES[case]
    ref = _build(n_nodes, calls, 7, 1)
    assert ref["src"].size > 1 << 16  # the sample sort runs
    for t in (2, 3, 8):
        got = _build(n_nodes, calls, 7, t)
        for k in ref:
            assert ref[k].dtype == got[k].dtype and ref[k].tobytes() == got[k].tobytes(), (t, k)


def test_node_and_value_arrays():
    rng = np.random.default_rng(5)
    n = 80_000
    perm = rng.permutation(500).astype(np.uint32)
    calls = [_c("fixed_indegree", (0, 500), (500, 200), n // 200, weight=("normal", 0.0, 1.0),
                delay=("uniform_int", 1, 9), src_idx=perm),
             _c("fixed_total_number", (0, 700), (0, 700), n, weight=("const", 1.0), delay=("const", 0.1),
                w_arr=rng.normal(size=n).astype(np.float32),
                d_arr=rng.uniform(0.0, 2.0, n).astype(np.float32))]
    ref = _build(700, calls, 3, 1)
    got = _build(700, calls, 3, 6)
    for k in ref:
        assert ref[k].tobytes() == got[k].tobytes(), k


def test_threads_setting_is_scoped():
    assert oracle.get_threads() == 1
    with oracle.threads(4):
        assert oracle.get_threads() == 4
    assert oracle.get_threads() == 1


def _lowbias32_inverse(y: int) -> int:
    """The inverse that C. Wellons publishes for lowbias32 (hash-prospector):
    multipliers 0x43021123 and 0x1d69e2a5, shift-xors undone step by step."""
    M = 0xFFFFFFFF
    y ^= y >> 16
    y = (y * 0x43021123) & M
    y ^= (y >> 15) ^ (y >> 30)
    y = (y * 0x1D69E2A5) & M
    y ^= y >> 16
    return y


def test_lowbias32_against_its_published_inverse():
    # The published inverse is independent of the forward constants in the
    # oracle: a wrong multiplier or shift there breaks the round trip.
    rng = np.random.default_rng(11)
    xs = [0, 1, 2, 0xFFFFFFFF, 0x80000000, 0x7FFFFFFF, 0x12345678, 0xDEADBEEF]
    xs += [int(v) for v in rng.integers(0, 1 << 32, 20_000, dtype=np.uint64)]
    for x in xs:
        assert _lowbias32_inverse(oracle.lowbias32(x)) == x, hex(x)
    # a bijection that is not the identity and moves low bits to high ones
    assert oracle.lowbias32(1) >> 16 != 0
    assert len({oracle.lowbias32(x) for x in range(4096)}) == 4096
