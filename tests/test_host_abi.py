"""CPU-only checks of the C-ABI library: it loads, exports every declared
symbol, and its pure host logic (Eq. (1) block planning, Connect validation
and counts of Sec. 2.1) behaves as specified.  No device work is done here."""
import ctypes
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

ng = pytest.importorskip("paper_2306_09855_amd.ng")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ng.LIB_PATH):
        pytest.skip("libng.so not built")
    return ng.lib()


def test_exports_every_declared_symbol(L):
    names = ng.declared_symbols()
    assert "ng_connect" in names and "ng_calibrate" in names and "ng_get_connections" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert not [n for n in names if not hasattr(ng, n)]


def test_version(L):
    assert "gfx950" in ng.ng_version()


def test_blocks_needed_fig1_golden(L):
    rows = np.loadtxt(os.path.join(HERE, "golden", "fig1_blocks.txt"), dtype=np.int64)
    for B, n_conns, n_blocks, n_new, n_newblocks, n_prev2 in rows:
        assert ng.ng_blocks_needed(int(n_conns), int(n_new), int(B), int(n_blocks)) == n_newblocks
        # Eq. (3): the new connections that precede block b = 2 fill the rest of block 1
        assert B * n_blocks - n_conns == n_prev2


@pytest.mark.parametrize("n_conns,n_new,B,n_blocks,expected", [
    (0, 0, 10, 0, 0),          # nothing to store
    (0, 1, 10, 0, 1),
    (0, 10, 10, 0, 1),         # exactly one full block
    (0, 11, 10, 0, 2),
    (5, 5, 10, 1, 0),          # fills the free slots of the last block
    (5, 6, 10, 1, 1),
    (20, 0, 10, 2, 0),
    (3, 1, 10, 4, 0),          # spare capacity: never negative
    (10**7 - 1, 2, 10**7, 1, 1),
    (300_000_000, 0, 1 << 24, 18, 0),
    (0, 300_000_000, 1 << 24, 0, 18),
])
def test_blocks_needed_eq1(L, n_conns, n_new, B, n_blocks, expected):
    assert ng.ng_blocks_needed(n_conns, n_new, B, n_blocks) == expected


def _count(n_nodes, rule, src, tgt, k=0, w=("normal", 0.5, 0.05), d=("uniform_int", 1, 20), h=0.1):
    return ng.ng_plan_count(n_nodes, ng.ng_range(*src), ng.ng_range(*tgt), ng.conn_spec(rule, k),
                            ng.syn_spec(w, d), h)


def test_plan_counts(L):
    assert _count(100, "one_to_one", (0, 10), (50, 10)) == 10
    assert _count(100, "all_to_all", (0, 7), (10, 9)) == 63
    assert _count(100, "fixed_indegree", (0, 7), (10, 9), 4) == 36
    assert _count(100, "fixed_outdegree", (0, 7), (10, 9), 4) == 28
    assert _count(100, "fixed_total_number", (0, 7), (10, 9), 12345) == 12345
    assert _count(100, "fixed_total_number", (0, 7), (10, 9), 0) == 0
    assert _count(100, "all_to_all", (0, 0), (10, 9)) == 0


@pytest.mark.parametrize("args,status", [
    ((100, "one_to_one", (0, 10), (50, 11)), ng.NG_ERR_INVALID_ARG),       # Eqs. (4)-(5) need N_s = N_t
    ((100, "all_to_all", (95, 10), (0, 5)), ng.NG_ERR_INVALID_ARG),        # range past the created nodes
    ((100, "fixed_indegree", (0, 0), (0, 5), 3), ng.NG_ERR_INVALID_ARG),   # no sources to draw from
    ((100, "fixed_outdegree", (0, 5), (0, 0), 3), ng.NG_ERR_INVALID_ARG),
    ((100, "fixed_total_number", (0, 5), (0, 0), 3), ng.NG_ERR_INVALID_ARG),
    ((100_000, "all_to_all", (0, 70_000), (0, 70_000)), ng.NG_ERR_TOO_LARGE),
])
def test_plan_errors(L, args, status):
    with pytest.raises(ng.NGError) as e:
        _count(*args)
    assert e.value.status == status


def test_spec_errors(L):
    bad = [
        dict(w=("normal", 0.5, -1.0)),
        dict(w=("uniform", 2.0, 1.0)),
        dict(w=("uniform_int", 1, 2)),
        dict(d=("uniform_int", 0, 5)),
        dict(d=("uniform_int", 1.5, 5)),
        dict(d=("uniform_int", 1, 40000)),
        dict(d=("normal", 1.0, 0.1)),
        dict(d=("const", 10000.0)),       # 100000 steps at h = 0.1
    ]
    for kw in bad:
        with pytest.raises(ng.NGError) as e:
            _count(100, "all_to_all", (0, 3), (0, 3), **kw)
        assert e.value.status == ng.NG_ERR_INVALID_ARG, kw


def test_autapse_multapse_flags(L):
    spec = ng.conn_spec("fixed_indegree", 3, allow_autapses=0)
    syn = ng.syn_spec(("const", 1.0), ("const", 1.0))
    # disjoint ranges: autapses cannot occur
    assert ng.ng_plan_count(10, ng.ng_range(0, 5), ng.ng_range(5, 5), spec, syn, 0.1) == 15
    # overlapping ranges: counts without the self-pairs
    assert ng.ng_plan_count(10, ng.ng_range(0, 5), ng.ng_range(3, 5), spec, syn, 0.1) == 15
    no_self = lambda rule, k=0: ng.conn_spec(rule, k, allow_autapses=0)  # noqa: E731
    assert ng.ng_plan_count(10, ng.ng_range(0, 5), ng.ng_range(3, 5), no_self("all_to_all"), syn, 0.1) == 23
    assert ng.ng_plan_count(10, ng.ng_range(2, 5), ng.ng_range(2, 5), no_self("one_to_one"), syn, 0.1) == 0
    assert ng.ng_plan_count(10, ng.ng_range(2, 5), ng.ng_range(3, 5), no_self("one_to_one"), syn, 0.1) == 5
    for rule, src, tgt in [("fixed_indegree", (4, 1), (3, 5)), ("fixed_outdegree", (3, 5), (4, 1)),
                           ("fixed_total_number", (4, 1), (4, 1))]:
        with pytest.raises(ng.NGError) as e:  # only autapses possible
            ng.ng_plan_count(10, ng.ng_range(*src), ng.ng_range(*tgt), no_self(rule, 3), syn, 0.1)
        assert e.value.status == ng.NG_ERR_INVALID_ARG
    # no multapses: distinct draws, at most as many as the candidates
    assert ng.ng_plan_count(10, ng.ng_range(0, 5), ng.ng_range(5, 5),
                            ng.conn_spec("fixed_indegree", 3, allow_multapses=0), syn, 0.1) == 15
    for rule, k, src, tgt in [("fixed_indegree", 6, (0, 5), (5, 5)), ("fixed_outdegree", 6, (0, 5), (5, 5)),
                              ("fixed_total_number", 26, (0, 5), (5, 5)),
                              ("fixed_indegree", 5, (0, 5), (0, 5))]:  # without autapses: 4 candidates
        with pytest.raises(ng.NGError) as e:
            ng.ng_plan_count(10, ng.ng_range(*src), ng.ng_range(*tgt),
                             ng.conn_spec(rule, k, allow_autapses=0 if src == tgt else 1, allow_multapses=0),
                             syn, 0.1)
        assert e.value.status == ng.NG_ERR_INVALID_ARG, rule


def test_arena_for_sizes():
    from paper_2306_09855_amd.network import arena_bytes_for
    assert arena_bytes_for(300_000_000, 77169, 30) > 2 * 14 * 300_000_000
    assert arena_bytes_for(0, 1) > 0


@pytest.mark.parametrize("n_conns,n_nodes,max_delay", [
    (300_000_000, 77_169, 30), (100_000, 2_000, 20), (154_000_000, 100_000, 50),
    (445_000_000, 1_000_000, 63), (2_000_000, 1 << 24, 7), (5, 2, 1), (1 << 20, 1 << 22, 31),
    (12_345, 3, 32767), (1 << 31, 77_169, 30)])
def test_calibration_plan(L, n_conns, n_nodes, max_delay):
    # the digits cover the key exactly (source bits + delay bits, Sec. 2.2),
    # each at most 9 bits; a record is packed into one word only when the
    # key bits not yet applied and a target index fit in 32 bits
    p = ng.ng_calibration_plan(n_conns, n_nodes, max_delay)
    sbits = max(n_nodes - 1, 0).bit_length()
    dbits = int(max_delay).bit_length()
    keybits = sbits + dbits
    if keybits > 27:
        assert p["msd"] == 0 and p["b1"] == 0
        return
    # the default takes it from 2^25 connections on, when the sub-buckets
    # average 256 connections or more and the possible keys 10 or more
    dense = n_conns * 512 >= (n_nodes << dbits) * 5120
    big = n_conns >= 1 << 25
    assert p["msd"] == (2 if big and n_conns >= 256 << (p["b1"] + p["b2"]) and dense else 1)
    assert p["b1"] + p["b2"] + p["b3"] == keybits
    assert all(1 <= p[k] <= 9 for k in ("b1", "b3")) and 0 <= p["b2"] <= 9
    tbits = max(sbits, 1)
    assert p["narrow_a"] == int(p["b2"] + p["b3"] + tbits <= 32)
    assert p["narrow_b"] == int(p["b3"] + tbits <= 32)
    assert p["wgs_c"] >= 1 and p["tpr"] >= 1


def test_calibration_plan_rejects(L):
    assert ng.ng_calibration_plan(0, 100, 5)["msd"] == 0
    assert ng.ng_calibration_plan(1000, 1, 1)["msd"] == 0     # a one-bit key: LSD
    with pytest.raises(ng.NGError):
        ng.ng_calibration_plan(1000, 10, 0)


def test_time_only_rejects(L):
    # no context, or a name longer than ng_kernel_time holds
    assert L.ng_time_only(None, b"msd_tiles_c") == ng.NG_ERR_INVALID_ARG
    assert L.ng_time_only(None, None) == ng.NG_ERR_INVALID_ARG
