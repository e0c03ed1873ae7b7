"""The fixed-scratch calibration (ng_calibrate_noalloc), for callers that
cannot allocate, against ng_calibrate through the C ABI.

Two calls in a row on fresh contexts, the second with a smaller input (the
fixed region keeps the first call's contents), each compared element by
element with ng_calibrate of the same network: sorted sources, targets,
delays and weights, group_ptr and group_start, all bit for bit (the same
kernels run on the same records).  A network whose scratch exceeds the
region is refused with NG_ERR_TOO_LARGE and the context is left as it was.
"""
import numpy as np
import pytest

from paper_2306_09855_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd import ng  # noqa: E402
from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402


def _calibrated(wl, noalloc: bool):
    with Network(wl.seed, wl.h, 1 << 16, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, 1 << 16)) as net:
        net.build(wl, calibrate=False)
        if noalloc:
            ng.ng_calibrate_noalloc(net.ctx)
        else:
            net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
        used = net.memory_stats()
    return out, gp, gs, used


def _same(a, b):
    out_a, gp_a, gs_a, _ = a
    out_b, gp_b, gs_b, _ = b
    for k in ("src", "tgt", "w", "delay"):
        assert out_a[k].dtype == out_b[k].dtype and np.array_equal(out_a[k].view(np.uint8),
                                                                    out_b[k].view(np.uint8)), k
    assert np.array_equal(gp_a, gp_b) and np.array_equal(gs_a, gs_b)


def test_two_calls_in_a_row_match_ng_calibrate():
    assert ng.ng_noalloc_scratch_bytes() == 64 << 20
    big = W.microcircuit(scale=0.07)        # ~1.5e6 connections, 18-bit keys: three digit passes
    small = W.two_pop_indegree(scale=0.45)  # ~2e4 connections, 15-bit keys: two passes
    assert big.n_syn > 1_000_000 and small.n_syn < big.n_syn
    for wl in (big, small):
        print(f"noalloc: {wl.name} n_syn={wl.n_syn}", flush=True)
        _same(_calibrated(wl, True), _calibrated(wl, False))


def test_too_large_is_refused_and_changes_nothing():
    wl = W.microcircuit(scale=0.11)  # ~3.6e6 connections: 24 B each exceed 64 MiB
    print(f"noalloc refusal: n_syn={wl.n_syn}", flush=True)
    with Network(wl.seed, wl.h, 1 << 20, arena_bytes_for(wl.n_syn, wl.n_nodes, wl.max_delay, 1 << 20)) as net:
        net.build(wl, calibrate=False)
        before = net.fetch(0, 1000)
        with pytest.raises(ng.NGError) as e:
            ng.ng_calibrate_noalloc(net.ctx)
        assert e.value.status == ng.NG_ERR_TOO_LARGE
        assert net.view().calibrated == 0
        after = net.fetch(0, 1000)
        for k in before:
            assert np.array_equal(before[k], after[k])
        net.calibrate()  # the ordinary path still works on the same context
        assert net.view().calibrated == 1
