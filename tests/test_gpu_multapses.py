"""GPU parity of the multapse prohibition (allow_multapses = 0; future work in
the Discussion), through the C ABI, against the CPU oracle: creation order and
calibrated arrays element by element, for fixed_indegree / fixed_outdegree
(keyed permutations per node, with and without autapses, K up to all
candidates) and fixed_total_number (a permutation of the pair index, up to all
pairs and over more than 2^32 pairs), in the plain and batched forms."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from parity import check_calibrated, check_creation_order

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09855_amd.network import Network  # noqa: E402

N_NODES = 100_000


def _call(rule, src, tgt, k, autapses=1, d=("uniform_int", 1, 30)):
    c = SimpleNamespace(rule=rule, src=src, tgt=tgt, k_or_n=k, weight=("normal", 0.5, 0.05), delay=d,
                        allow_autapses=autapses, allow_multapses=0)
    c.n_syn = lambda: oracle.count(c)
    return c


CASES = {
    "indegree": [_call("fixed_indegree", (0, 3000), (3000, 200), 150)],
    "indegree_all_sources": [_call("fixed_indegree", (0, 97), (200, 50), 97)],
    "indegree_no_autapses_all": [_call("fixed_indegree", (10, 64), (10, 64), 63, autapses=0)],
    "outdegree": [_call("fixed_outdegree", (0, 200), (500, 5000), 321, d=("uniform", 0.1, 4.0))],
    "outdegree_no_autapses": [_call("fixed_outdegree", (0, 400), (100, 400), 99, autapses=0)],
    "total": [_call("fixed_total_number", (0, 300), (300, 200), 40_000)],
    "total_all_pairs_no_autapses": [_call("fixed_total_number", (0, 40), (20, 40), 40 * 40 - 20, autapses=0)],
    "total_wide_pair_space": [_call("fixed_total_number", (0, 100_000), (0, 60_000), 50_000)],  # 6e9 pairs
    # every pair, or all but one, with a count that is not a multiple of 4: the lanes past the
    # call's end must not walk from an index outside the pair space
    "total_all_pairs_ragged": [_call("fixed_total_number", (0, 7), (100, 9), 63)],
    "total_all_but_one_ragged": [_call("fixed_total_number", (0, 7), (100, 9), 62)],
    "total_all_pairs_no_autapses_ragged": [_call("fixed_total_number", (0, 7), (3, 9), 59, autapses=0)],
}


@pytest.mark.parametrize("batched", [False, True], ids=["plain", "batched"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_no_multapses_match_oracle(name, batched):
    calls = CASES[name]
    ref = oracle.build_network(13, 0.1, N_NODES, calls)
    with Network(13, 0.1, 1 << 16, 256 << 20) as net:
        net.create(N_NODES)
        if batched:
            net.connect_batch(calls)
        else:
            for c in calls:
                net.connect(c)
        # raises if a permutation walk started at or above its bound or reached its step cap
        net.sync()
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
        net.sync()
    check_creation_order(created, ref, calls)
    check_calibrated(out, gp, gs, ref, calls)
    pairs = created["src"].astype(np.int64) * N_NODES + created["tgt"]
    assert np.unique(pairs).size == pairs.size
