"""Full-size parity, every element: the benchmark's networks built on the GPU
in the launch configuration the benchmark times, compared with the oracle
(run with all host cores; its threaded mode is byte-identical to the
single-thread mode, tests/test_oracle_threads.py) on every connection.

  * microcircuit: 77,169 nodes, 64 fixed_total_number calls, 3.0e8 synapses,
    one ng_connect per call, then ng_calibrate (Sec. 2.1, 2.2);
  * two-population network: E and I of 50,000 nodes, four calls with four
    rules, 1.54e8 synapses;
  * batched form: 4,096 uneven calls of mixed rules over 1e6 nodes (~4.3e8
    synapses) through one ng_connect_batch.

Creation order is compared call by call (sources, targets, delays bit for
bit; weights within the bound of tests/parity.py), then the calibrated
arrays in chunks against the oracle's stable order, then group_ptr (Eq. (14))
and group_start.  The largest relative weight error is printed next to the
bound.  Host memory stays at about 40 bytes per synapse.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W
from parity import WEIGHT_RTOL, check_equal, check_weights

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd.network import Network, arena_bytes_for  # noqa: E402

CHUNK = 1 << 25


def _threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _compare_full(wl, batched=False, block_size=1 << 24):
    n = wl.n_syn
    starts = np.concatenate([[0], np.cumsum([c.n_syn() for c in wl.calls])]).astype(np.int64)
    net = Network(wl.seed, wl.h, block_size, arena_bytes_for(n, wl.n_nodes, wl.max_delay, block_size))
    src = np.empty(n, np.uint32)
    tgt = np.empty(n, np.uint32)
    w = np.empty(n, np.float64)
    d = np.empty(n, np.int32)
    base = np.empty(n, np.float64)
    worst = 0.0
    try:
        net.build(wl, batched=batched, calibrate=False)
        with oracle.threads(_threads()):
            for c, call in enumerate(wl.calls):
                a, b = int(starts[c]), int(starts[c + 1])
                if a == b:
                    continue
                s_, t_, w_, d_ = oracle.connect(wl.seed, wl.h, c, call)
                src[a:b], tgt[a:b], w[a:b], d[a:b] = s_, t_, w_, d_
                base[a:b] = float(call.weight[1])
                g = net.fetch(a, b - a)
                check_equal(g["src"], s_, f"call {c} src")
                check_equal(g["tgt"], t_, f"call {c} tgt")
                check_equal(g["delay"], d_, f"call {c} delay")
                check_weights(g["w"], w_, base[a:b], f"call {c} w")
                nz = w_ != 0
                if nz.any():
                    worst = max(worst, float(np.max(np.abs(g["w"][nz].astype(np.float64) - w_[nz]) / np.abs(w_[nz]))))
            net.calibrate()
            perm, gp_ref, gs_ref = oracle.calibrate(wl.n_nodes, src, d)
        for a in range(0, n, CHUNK):
            b = min(n, a + CHUNK)
            p = perm[a:b].astype(np.int64)
            g = net.fetch(a, b - a)
            check_equal(g["src"], src[p], f"sorted src [{a}, {b})")
            check_equal(g["tgt"], tgt[p], f"sorted tgt [{a}, {b})")
            check_equal(g["delay"], d[p], f"sorted delay [{a}, {b})")
            check_weights(g["w"], w[p], base[p], f"sorted w [{a}, {b})")
        gp, gs = net.group_index()
        check_equal(gp, gp_ref, "group_ptr")
        check_equal(gs, gs_ref, "group_start")
    finally:
        net.close()
        torch.cuda.empty_cache()
    print(f"\n{wl.name}: {n} synapses, {gs.size - 1} groups equal to the oracle; "
          f"max |dw|/|w| = {worst:.3g} (bound {WEIGHT_RTOL:g} x (|mean| + |w - mean|))")
    return worst


def test_microcircuit_3e8_every_synapse():
    wl = W.microcircuit()
    assert wl.n_syn == 300_000_000
    _compare_full(wl)


def test_two_population_network_every_synapse():
    wl = W.two_pop_mixed()
    assert wl.n_syn == 154_000_000
    _compare_full(wl)


def test_batched_4096_calls_every_synapse():
    wl = W.batch_mixed()
    assert len(wl.calls) == 4096
    _compare_full(wl, batched=True)
