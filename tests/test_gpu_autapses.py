"""GPU parity of the autapse prohibition (allow_autapses = 0; a flag the
paper names as future work, Discussion), through the C ABI, against the CPU
oracle: creation order and calibrated arrays element by element, for every
rule with partly and fully overlapping ranges, in the plain and batched forms.
The 64th-attempt fallback of fixed_total_number is not reached by these
inputs (its probability is at most 2^-63 per synapse)."""
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

N_NODES = 2000


def _call(rule, src, tgt, k, w=("normal", 0.5, 0.05), d=("uniform_int", 1, 30)):
    c = SimpleNamespace(rule=rule, src=src, tgt=tgt, k_or_n=k, weight=w, delay=d, allow_autapses=0)
    c.n_syn = lambda: oracle.count(c)
    return c


CASES = {
    "one_to_one_shifted": [_call("one_to_one", (100, 500), (150, 500), 0)],
    "one_to_one_same": [_call("one_to_one", (100, 500), (100, 500), 0),
                        _call("fixed_total_number", (0, 50), (60, 50), 1000)],
    "all_to_all_partial": [_call("all_to_all", (0, 120), (80, 100), 0)],
    "all_to_all_same": [_call("all_to_all", (10, 150), (10, 150), 0)],
    "all_to_all_one_target": [_call("all_to_all", (0, 200), (57, 1), 0)],
    "indegree": [_call("fixed_indegree", (0, 400), (300, 400), 23)],
    "indegree_same": [_call("fixed_indegree", (500, 64), (500, 64), 97)],
    "outdegree": [_call("fixed_outdegree", (300, 400), (0, 400), 29)],
    "total_partial": [_call("fixed_total_number", (0, 700), (600, 700), 200_003)],
    "total_three_nodes": [_call("fixed_total_number", (7, 3), (7, 3), 50_000)],
}


def _run(calls, batched):
    with Network(31, 0.1, 1 << 16, 256 << 20) as net:
        net.create(N_NODES)
        if batched:
            net.connect_batch(calls)
        else:
            for c in calls:
                net.connect(c)
        created = net.fetch()
        net.calibrate()
        out = net.fetch()
        gp, gs = net.group_index()
    return created, out, gp, gs


@pytest.mark.parametrize("batched", [False, True], ids=["plain", "batched"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_no_autapses_match_oracle(name, batched):
    calls = CASES[name]
    ref = oracle.build_network(31, 0.1, N_NODES, calls)
    created, out, gp, gs = _run(calls, batched)
    check_creation_order(created, ref, calls)
    check_calibrated(out, gp, gs, ref, calls)
    assert not np.any(created["src"] == created["tgt"])
