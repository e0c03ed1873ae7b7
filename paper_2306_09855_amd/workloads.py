"""Seeded synthetic workloads: node populations and Connect-call lists.

This module holds no arithmetic of the method.  It only decides which nodes
are created and which Connect calls are issued, with which rule, sizes and
weight/delay specifications.  Both the GPU path and the CPU oracle consume the
same lists.

Workloads (shapes follow the networks of Sec. 2.4 of Golosio et al.):

* ``two_pop_indegree``   -- two populations of 1,000 nodes, A->B fixed_indegree
  K=100, Normal(0.5, 0.05) weights, delays uniform in {1..20} steps (1e5 synapses).
* ``two_pop_mixed``      -- the two-population scaling network: E and I of 50,000
  nodes, E->E fixed_indegree K=1000, E->I fixed_outdegree K=1000, I->E
  fixed_total_number 5e7, I->I all_to_all on the first 2,000 x 2,000 nodes
  (1.54e8 synapses), delays {1..50}.
* ``microcircuit``       -- eight populations of the cortical-microcircuit sizes
  (77,169 nodes), 64 fixed_total_number calls whose counts come from a seeded
  8x8 table of probabilities in [0, 0.15] scaled to 3.0e8 synapses in total;
  inhibitory source populations get Normal(-0.5, 0.05) weights; delays {1..30}.
  The real connectivity table is not reproduced: this is a stand-in with the
  same population sizes, rule and synapse count.
* ``batch_mixed``        -- 4,096 calls of log-uniform size in [1e2, 1e6], mixed
  rules, random ranges inside 1e6 nodes, delays {1..63}.

``scale`` shrinks a workload (population sizes and synapse counts) for tests
that must finish on the CPU oracle in seconds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RULES = ("one_to_one", "all_to_all", "fixed_indegree", "fixed_outdegree", "fixed_total_number")

MICROCIRCUIT_SIZES = (20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948)
MICROCIRCUIT_INHIBITORY = (1, 3, 5, 7)


@dataclass(frozen=True)
class Call:
    rule: str
    src: tuple            # (first node, count)
    tgt: tuple            # (first node, count)
    k_or_n: int = 0       # K for in/out-degree, N for fixed_total_number
    weight: tuple = ("normal", 0.5, 0.05)     # ("const", a) | ("normal", mean, sd) | ("uniform", lo, hi)
    delay: tuple = ("uniform_int", 1, 20)     # ("const", ms) | ("uniform_int", lo, hi) | ("uniform", lo_ms, hi_ms)

    def n_syn(self) -> int:
        ns, nt, k = self.src[1], self.tgt[1], self.k_or_n
        return {"one_to_one": ns, "all_to_all": ns * nt, "fixed_indegree": nt * k,
                "fixed_outdegree": ns * k, "fixed_total_number": k}[self.rule]


@dataclass
class Workload:
    name: str
    seed: int
    populations: list
    calls: list
    h: float = 0.1
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(sum(self.populations))

    @property
    def n_syn(self) -> int:
        return int(sum(c.n_syn() for c in self.calls))

    @property
    def max_delay(self) -> int:
        m = 1
        for c in self.calls:
            if c.delay[0] == "uniform_int":
                m = max(m, int(c.delay[2]))
        return m


def two_pop_indegree(seed: int = 12345, scale: float = 1.0) -> Workload:
    n = max(2, int(round(1000 * scale)))
    k = max(1, int(round(100 * scale)))
    calls = [Call("fixed_indegree", (0, n), (n, n), k, ("normal", 0.5, 0.05), ("uniform_int", 1, 20))]
    return Workload("two_pop_indegree", seed, [n, n], calls)


def two_pop_mixed(seed: int = 12345, scale: float = 1.0) -> Workload:
    npop = max(4, int(round(50000 * scale)))
    k = max(1, int(round(1000 * scale)))
    ntot = max(1, int(round(5e7 * scale * scale)))
    sub = max(1, min(npop, int(round(2000 * scale))))
    E, I = (0, npop), (npop, npop)
    w, d = ("normal", 0.5, 0.05), ("uniform_int", 1, 50)
    calls = [
        Call("fixed_indegree", E, E, k, w, d),
        Call("fixed_outdegree", E, I, k, w, d),
        Call("fixed_total_number", I, E, ntot, w, d),
        Call("all_to_all", (npop, sub), (npop, sub), 0, w, d),
    ]
    return Workload("two_pop_mixed", seed, [npop, npop], calls)


def microcircuit_table(total: int, sizes=MICROCIRCUIT_SIZES, table_seed: int = 3):
    """Synapse counts n_ij for source pop i -> target pop j.

    p_ij ~ U[0, 0.15] from a seeded generator; n_ij proportional to
    p_ij * N_i * N_j, scaled to sum exactly to ``total`` by the largest
    remainder method (ties go to the lower flat index)."""
    rng = np.random.default_rng(table_seed)
    p = rng.uniform(0.0, 0.15, size=(len(sizes), len(sizes)))
    N = np.asarray(sizes, dtype=np.float64)
    raw = p * N[:, None] * N[None, :]
    ideal = raw / raw.sum() * total
    base = np.floor(ideal).astype(np.int64)
    rem = total - int(base.sum())
    frac = (ideal - base).ravel()
    order = sorted(range(frac.size), key=lambda f: (-frac[f], f))
    flat = base.ravel()
    for f in order[:rem]:
        flat[f] += 1
    return flat.reshape(base.shape)


def microcircuit(seed: int = 12345, scale: float = 1.0, total: int | None = None) -> Workload:
    sizes = [max(1, int(round(s * scale))) for s in MICROCIRCUIT_SIZES]
    if total is None:
        total = int(round(3.0e8 * scale * scale))
    counts = microcircuit_table(total, sizes)
    firsts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(int)
    calls = []
    for i in range(len(sizes)):
        w = ("normal", -0.5, 0.05) if i in MICROCIRCUIT_INHIBITORY else ("normal", 0.5, 0.05)
        for j in range(len(sizes)):
            calls.append(Call("fixed_total_number", (int(firsts[i]), sizes[i]),
                              (int(firsts[j]), sizes[j]), int(counts[i, j]), w,
                              ("uniform_int", 1, 30)))
    return Workload("microcircuit", seed, sizes, calls)


def batch_mixed(seed: int = 12345, n_calls: int = 4096, n_nodes: int = 1_000_000,
                lo_exp: float = 2.0, hi_exp: float = 6.0, gen_seed: int = 4) -> Workload:
    """Uneven Connect calls for the batched form.

    Per call: a target size n = floor(10^U(lo_exp, hi_exp)) and a rule drawn
    uniformly.  Ranges are random inside ``n_nodes``:
      one_to_one      N_s = N_t = min(n, n_nodes)
      all_to_all      N_s = ceil(sqrt(n)), N_t = ceil(n / N_s)
      fixed_indegree  N_t = floor(10^U(0, log10 n)), K = ceil(n / N_t), N_s log-uniform
      fixed_outdegree N_s = floor(10^U(0, log10 n)), K = ceil(n / N_s), N_t log-uniform
      fixed_total     N_s, N_t log-uniform, N = n
    """
    rng = np.random.default_rng(gen_seed)
    calls = []

    def logu(hi):
        return max(1, min(n_nodes, int(10 ** rng.uniform(0.0, math.log10(max(hi, 1)) + 1e-12))))

    def start(cnt):
        return int(rng.integers(0, n_nodes - cnt + 1))

    for _ in range(n_calls):
        n = int(10 ** rng.uniform(lo_exp, hi_exp))
        rule = RULES[int(rng.integers(0, 5))]
        if rule == "one_to_one":
            ns = nt = min(n, n_nodes)
            k = 0
        elif rule == "all_to_all":
            ns = int(math.ceil(math.sqrt(n)))
            nt = int(math.ceil(n / ns))
            k = 0
        elif rule == "fixed_indegree":
            nt = logu(n)
            k = int(math.ceil(n / nt))
            ns = logu(n_nodes)
        elif rule == "fixed_outdegree":
            ns = logu(n)
            k = int(math.ceil(n / ns))
            nt = logu(n_nodes)
        else:
            ns, nt, k = logu(n_nodes), logu(n_nodes), n
        calls.append(Call(rule, (start(ns), ns), (start(nt), nt), k,
                          ("normal", 0.5, 0.05), ("uniform_int", 1, 63)))
    return Workload("batch_mixed", seed, [n_nodes], calls)


def by_name(name: str, **kw) -> Workload:
    return {"two_pop_indegree": two_pop_indegree, "two_pop_mixed": two_pop_mixed,
            "microcircuit": microcircuit, "batch_mixed": batch_mixed}[name](**kw)


@dataclass
class Episode:
    """One model-building session of the serving trace."""
    slot: int
    seed: int
    n_nodes: int
    calls: list
    times: list          # arrival times (s) of: create_nodes, each connect, calibrate, close

    @property
    def n_syn(self) -> int:
        return int(sum(c.n_syn() for c in self.calls))


def serving_trace(n_slots: int = 32, episodes_per_slot: int = 3, rate: float = 2000.0,
                  lo_exp: float = 3.0, hi_exp: float = 7.0, gen_seed: int = 5,
                  burst: bool = False) -> list:
    """Episodes of the serving workload.

    Each of ``n_slots`` clients runs ``episodes_per_slot`` sessions back to back:
    create floor(10^U(4,6)) nodes, M ~ U{4..32} Connect calls of log-uniform
    size in [10^lo_exp, 10^hi_exp] with mixed rules inside the session's nodes
    (as ``batch_mixed``), calibrate, close.  Requests of a client arrive as a
    Poisson process of rate ``rate / n_slots``; with ``burst`` every request
    arrives at time 0 (a backlog that measures capacity)."""
    rng = np.random.default_rng(gen_seed)
    out = []
    for slot in range(n_slots):
        t = 0.0
        for e in range(episodes_per_slot):
            n_nodes = int(10 ** rng.uniform(4.0, 6.0))
            m = int(rng.integers(4, 33))
            sub = batch_mixed(seed=0, n_calls=m, n_nodes=n_nodes, lo_exp=lo_exp, hi_exp=hi_exp,
                              gen_seed=int(rng.integers(1 << 31)))
            times = []
            for _ in range(m + 3):
                if not burst:
                    t += rng.exponential(n_slots / rate)
                times.append(t)
            out.append(Episode(slot, int(rng.integers(1, 1 << 62)), n_nodes, sub.calls, times))
    return out
