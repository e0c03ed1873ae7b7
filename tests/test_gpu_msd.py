"""GPU parity of the most-significant-digit calibration (the default radix
form for one large context, forced here with NG_CALIB_RADIX_MSD so that
small cases take it too): the stable order by (source, delay) and the group
index of Sec. 2.2, Eq. (14), against the oracle element by element, for every
digit geometry the plan can take, and bit for bit against the LSD form.

Geometries (checked through ng_calibration_plan before each run):
  * one scatter pass (b2 = 0) and two (b2 > 0);
  * records packed into one word after both scatters, only after the second,
    or after neither (many nodes: wide target indices);
  * sub-buckets larger than one LDS piece (heavy keys: a few sources, one
    delay), empty sub-buckets (sparse sources), ragged tails, one record;
  * range counts from 1 to more ranges than tiles; 2^16-connection blocks;
  * a first digit that reaches into the delay bits.
"""
import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W
from parity import check_calibrated, check_creation_order

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd import ng  # noqa: E402
from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402


def _run(wl, block_size=0, calibration="msd", ranges=None):
    B = block_size or (1 << 24)
    with Network(wl.seed, wl.h, block_size, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B)) as net:
        net.set_calibration(calibration)
        if ranges is not None:
            net.tune(9, ranges)
        net.build(wl, calibrate=False)
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    return created, out, gp, gs


def _plan(wl, ranges=1024):
    return ng.ng_calibration_plan(wl.n_syn, wl.n_nodes, wl.max_delay, ranges)


def _vs_oracle(wl, **kw):
    ref = oracle.build_network(wl.seed, wl.h, wl.n_nodes, wl.calls)
    created, out, gp, gs = _run(wl, **kw)
    check_creation_order(created, ref, wl.calls)
    check_calibrated(out, gp, gs, ref, wl.calls)


def _ftn(name, pops, src, tgt, n, delay=("uniform_int", 1, 30), seed=2718):
    return W.Workload(name, seed, pops, [W.Call("fixed_total_number", src, tgt, n, ("normal", 0.5, 0.05), delay)])


def test_one_scatter_pass():
    wl = W.two_pop_indegree()
    p = _plan(wl)
    assert p["msd"] >= 1 and p["b2"] == 0
    _vs_oracle(wl)


def test_two_scatter_passes_packed():
    wl = W.two_pop_mixed(scale=0.1)
    p = _plan(wl)
    assert p["msd"] >= 1 and p["b2"] > 0 and p["narrow_a"] == 1
    _vs_oracle(wl, block_size=1 << 16)


def test_microcircuit_two_scatter_passes():
    # 11,575 nodes and delays up to 30: a 19-bit key, two scatter passes
    wl = W.microcircuit(scale=0.15)
    p = _plan(wl)
    assert p["msd"] >= 1 and p["b2"] > 0 and p["narrow_a"] == 1
    _vs_oracle(wl)


def test_wide_after_first_scatter():
    # 2^20 nodes and delays up to 63: the key bits left after D1 plus a 20-bit
    # target do not fit one word, those left after D2 do
    wl = _ftn("wide_a", [1 << 20], (0, 1 << 20), (0, 1 << 20), 400_001, ("uniform_int", 1, 63))
    p = _plan(wl)
    assert p["msd"] >= 1 and p["b2"] > 0 and p["narrow_a"] == 0 and p["narrow_b"] == 1
    _vs_oracle(wl)


def test_wide_after_both_scatters():
    # 2^24 nodes (24-bit targets) and delays up to 7: a 27-bit key, no packing
    wl = _ftn("wide_ab", [1 << 24], (0, 1 << 24), (0, 1 << 24), 300_007, ("uniform_int", 1, 7))
    p = _plan(wl)
    assert p["msd"] >= 1 and p["narrow_a"] == 0 and p["narrow_b"] == 0
    _vs_oracle(wl)


def test_wide_and_sparse():
    # 3,001 connections over 2^24 nodes: unpacked records, almost every
    # bucket and sub-bucket empty
    wl = _ftn("wide_sparse", [1 << 24], (0, 1 << 24), (0, 1 << 24), 3_001, ("uniform_int", 1, 1))
    p = _plan(wl)
    assert p["msd"] >= 1 and p["narrow_b"] == 0
    _vs_oracle(wl)


@pytest.mark.parametrize("n_src,n", [(1, 70_003), (3, 250_000)])
def test_heavy_keys(n_src, n):
    # every connection from one or three sources with one delay: sub-buckets
    # of up to 2.5e5 records, sorted in several LDS pieces; 200,000 target
    # nodes keep the key wide enough for two scatter passes
    pops = [n_src, 200_000]
    wl = _ftn("heavy", pops, (0, n_src), (n_src, 200_000), n, ("uniform_int", 4, 4))
    wl.calls.append(W.Call("fixed_total_number", (0, n_src + 200_000), (0, 5), 9_999, ("normal", -0.5, 0.05),
                           ("uniform_int", 1, 9)))
    _vs_oracle(wl)


def test_sparse_sources_and_single_record():
    # sources spread thinly over 3e5 nodes leave most sub-buckets empty; a
    # second context holds a single connection
    wl = _ftn("sparse", [300_000], (0, 300_000), (0, 50), 20_000, ("uniform_int", 1, 30))
    assert _plan(wl)["b2"] > 0
    _vs_oracle(wl)
    one = _ftn("one", [3, 4], (0, 3), (3, 4), 1, ("uniform_int", 2, 5))
    _vs_oracle(one)


@pytest.mark.parametrize("pops,max_delay,n", [((20, 30), 1000, 600_001), ((8, 8), 30_000, 900_001)])
def test_delay_bits_in_first_digit(pops, max_delay, n):
    # 50 or 16 nodes with delays of up to 10 or 15 bits: the first digit
    # reaches into the delay bits, so the first count reads delays too; one
    # scatter pass, then two; 2^16-connection blocks, so that ranges of
    # 10,240-record tiles cross block ends
    a, b = pops
    wl = W.Workload("delay_d1", 31, [a, b], [W.Call("fixed_total_number", (0, a), (a, b), n, ("normal", 0.5, 0.05),
                                                    ("uniform_int", 1, max_delay))])
    p = _plan(wl)
    assert p["msd"] >= 1 and p["b2"] + p["b3"] < max_delay.bit_length()
    _vs_oracle(wl, block_size=1 << 16)


@pytest.mark.parametrize("ranges", [1, 3, 100_000])
def test_range_counts(ranges):
    wl = W.microcircuit(scale=0.03)
    assert _plan(wl, ranges)["msd"] >= 1
    _vs_oracle(wl, ranges=ranges)


def test_mixed_rules_and_batches():
    wl = W.batch_mixed(n_calls=200, n_nodes=300_000, lo_exp=1.0, hi_exp=4.0, gen_seed=11)
    assert _plan(wl)["msd"] >= 1
    _vs_oracle(wl)


def _same(a, b):
    for x, y in zip(a[:2], b[:2]):
        for k in ("src", "tgt", "delay"):
            assert np.array_equal(x[k], y[k]), k
        assert np.array_equal(x["w"].view(np.uint32), y["w"].view(np.uint32))
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_equals_lsd_many_blocks():
    # 3.7e7 connections in 2^16-connection blocks: 561 output blocks, more
    # than the in-LDS block table holds; the LSD form is the reference here
    # (it is checked against the oracle in the other parity tests)
    wl = W.microcircuit(scale=0.35)
    assert wl.n_syn > 512 * (1 << 16)
    _same(_run(wl, block_size=1 << 16), _run(wl, block_size=1 << 16, calibration="lsd"))


def test_equals_lsd_two_pop_mixed():
    wl = W.two_pop_mixed(scale=0.1)
    assert _plan(wl)["msd"] >= 1
    _same(_run(wl), _run(wl, calibration="lsd"))


def test_many_heavy_sub_buckets():
    # eight single sources far apart, 40,000 connections each with one of two
    # delays: eight sub-buckets larger than one LDS load, sorted in pieces by
    # several workgroups at once, next to ordinary tiles
    pops = [8_000, 200_000]
    calls = [W.Call("fixed_total_number", (1000 * k, 1), (8_000, 200_000), 40_000 + k,
                    ("normal", 0.5, 0.05), ("uniform_int", 3, 4)) for k in range(8)]
    calls.append(W.Call("fixed_total_number", (0, 8_000), (8_000, 200_000), 60_000, ("normal", -0.5, 0.05),
                        ("uniform_int", 1, 7)))
    wl = W.Workload("heavy8", 99, pops, calls)
    assert _plan(wl)["b2"] > 0
    _vs_oracle(wl)


def _kernels_used(wl, calibration):
    B = 1 << 24
    with Network(wl.seed, wl.h, 0, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B)) as net:
        net.set_calibration(calibration)
        net.build(wl, calibrate=False)
        ng.ng_enable_timing(net.ctx, True)
        ng.ng_read_timing(net.ctx, reset=True)
        net.calibrate()
        net.sync()
        names = set(ng.ng_read_timing(net.ctx, reset=True))
    return names


def test_time_only_brackets_one_kernel():
    # with ng_time_only, only the named launches are timed; the arrays are
    # those of the build with every launch timed
    wl = W.microcircuit(scale=0.35)
    B = 1 << 24
    outs = []
    for only in ("msd_tiles_c", None):
        with Network(wl.seed, wl.h, 0, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, B)) as net:
            ng.ng_time_only(net.ctx, only)
            ng.ng_enable_timing(net.ctx, True)
            ng.ng_read_timing(net.ctx, reset=True)
            net.build(wl)
            names = ng.ng_read_timing(net.ctx, reset=True)
            outs.append((net.fetch(), *net.group_index()))
        if only:
            assert set(names) == {"msd_tiles_c"} and names["msd_tiles_c"][0] == 1
        else:
            assert {"generate_batch", "msd_scatter_a", "msd_tiles_c", "msd_groups"} <= set(names)
    a, b = outs
    for k in ("src", "tgt", "delay"):
        assert np.array_equal(a[0][k], b[0][k]), k
    assert np.array_equal(a[0]["w"].view(np.uint32), b[0]["w"].view(np.uint32))
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    with Network(wl.seed, wl.h, 0, 1 << 26) as net:
        with pytest.raises(ng.NGError):
            ng.ng_time_only(net.ctx, "x" * 24)


def test_default_form_choice():
    # the default radix calibration sorts most-significant digit first from
    # 2^25 connections on, when the sub-buckets average 256 connections or
    # more and the possible keys 10 or more, else by LSD passes
    big = W.microcircuit(scale=0.35)  # 3.7e7 connections, 42 per possible key
    assert _plan(big)["msd"] == 2
    small = W.microcircuit(scale=0.1)  # 3e6 connections
    assert _plan(small)["msd"] == 1
    assert "downsweep" in _kernels_used(small, "radix")
    names = _kernels_used(big, "radix")
    assert "msd_scatter_a" in names and "downsweep" not in names
    sparse = _ftn("sparse_default", [1 << 20], (0, 1 << 20), (0, 1 << 20), 5_000, ("uniform_int", 1, 63))
    assert _plan(sparse)["msd"] == 1
    names = _kernels_used(sparse, "radix")
    assert "downsweep" in names and not any(n.startswith("msd") for n in names)
    assert "downsweep" in _kernels_used(big, "lsd")
    low_density = W.microcircuit(scale=0.05)  # 6 connections per possible key
    assert _plan(low_density)["msd"] == 1
    assert "downsweep" in _kernels_used(low_density, "radix")
