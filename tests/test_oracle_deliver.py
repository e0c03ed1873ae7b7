"""Pin of the oracle's spike buffer and delivery (Sec. 2.3) against the plain
definition, computed from the creation-order arrays with no groups, queues or
calibration: the input of target t at step T is the sum, over spikes (node i,
step T0, multiplicity m) and over connections c from i to t with
T0 + delay_c == T, of w_c * m.  Covers nodes that spike every step (the
queue at its longest), nodes without outgoing connections, multiplicities
above one and delays up to 20 steps."""
import numpy as np
import pytest

import oracle
from paper_2306_09855_amd import workloads as W


def _spikes(rng, n_nodes, n_steps, p, always=()):
    out = []
    for _ in range(n_steps):
        nodes = np.nonzero(rng.random(n_nodes) < p)[0]
        nodes = np.union1d(nodes, np.asarray(always, np.int64))
        out.append((nodes.astype(np.uint32), rng.integers(1, 4, nodes.size).astype(np.uint32)))
    return out


def _definition(n_nodes, net, spikes):
    src, tgt, w, d = net["src"].astype(np.int64), net["tgt"].astype(np.int64), net["w"], net["delay"].astype(np.int64)
    out = np.zeros((len(spikes), n_nodes))
    for T0, (nodes, mult) in enumerate(spikes):
        m = np.zeros(n_nodes)
        m[nodes.astype(np.int64)] = mult
        sel = m[src] > 0
        T = T0 + d[sel]
        ok = T < len(spikes)
        np.add.at(out, (T[ok], tgt[sel][ok]), (w[sel] * m[src[sel]])[ok])
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_delivery_matches_definition(seed):
    calls = [
        W.Call("fixed_total_number", (0, 40), (40, 60), 3000, ("normal", 0.5, 0.2), ("uniform_int", 1, 20)),
        W.Call("fixed_indegree", (40, 60), (0, 40), 7, ("uniform", -1.0, 1.0), ("uniform_int", 1, 5)),
        W.Call("all_to_all", (90, 5), (0, 100), 0, ("const", 0.25), ("const", 1.3)),
    ]
    n_nodes = 120  # nodes 100..119 have no outgoing connections
    net = oracle.build_network(seed, 0.1, n_nodes, calls)
    rng = np.random.default_rng(seed)
    spikes = _spikes(rng, n_nodes, 70, 0.08, always=(3, 45, 92, 110))
    got = oracle.deliver(n_nodes, net, spikes)
    ref = _definition(n_nodes, net, spikes)
    scale = np.abs(net["w"]).max() * 3 * 100
    assert np.abs(got - ref).max() <= 1e-12 * scale
    assert np.abs(ref).max() > 0


def test_no_spikes_no_input():
    calls = [W.Call("all_to_all", (0, 10), (0, 10), 0, ("const", 1.0), ("const", 0.1))]
    net = oracle.build_network(4, 0.1, 10, calls)
    empty = [(np.zeros(0, np.uint32), np.zeros(0, np.uint32))] * 5
    assert not oracle.deliver(10, net, empty).any()
