"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method itself: it only builds graphs (symmetric int32
CSR with ascending neighbour lists) and workload recipes.

* ``planted_partition``: an LFR-style planted-partition graph written from the LFR method
  description (power-law degrees, power-law community sizes, mixing parameter mu,
  configuration-model wiring inside and between communities, self-loops and multi-edges
  dropped, node ids permuted). It stands in for the networkx LFR graphs and the real
  datasets the paper measures on (section 5.2), none of which are available here.
* the small graphs drawn in the paper (Fig. 1, Fig. 3, the crossover/mutation example of
  the appendix) and a few edge-case shapes (star, path, clique, isolated nodes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray          # int32[n+1]
    col: np.ndarray              # int32[2m], ascending within each row
    membership: np.ndarray | None = None   # planted community of every node (if any)
    info: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2

    @property
    def deg(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def csr_from_edges(n: int, edges) -> Graph:
    """Symmetric CSR of an undirected simple graph given as (u, v) pairs. Self-loops and
    duplicate edges are dropped."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    assert row_ptr[-1] < 2**31
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32))


# ------------------------------------------------------------------------------------------
# Graphs drawn in the paper
# ------------------------------------------------------------------------------------------
def _clique(nodes):
    return [(a, b) for i, a in enumerate(nodes) for b in nodes[i + 1:]]


def fig1_graph() -> Graph:
    """Fig. 1 (introduction): two 5-node cliques joined by one bridge edge. Nodes 0-4 and
    5-9; the bridge joins node 0 (the angle-0 node of the first clique) to node 7 (the
    angle-144 node of the second)."""
    edges = _clique(list(range(5))) + _clique(list(range(5, 10))) + [(0, 7)]
    g = csr_from_edges(10, edges)
    g.membership = np.array([0] * 5 + [1] * 5, dtype=np.int32)
    return g


def fig3_graph() -> Graph:
    """Fig. 3 toy network (section 4, solution representation): three 4-cliques {1..4},
    {5..8}, {9..12} and the bridges 4-5, 4-10, 5-10 (paper ids minus one here)."""
    edges = (_clique([0, 1, 2, 3]) + _clique([4, 5, 6, 7]) + _clique([8, 9, 10, 11])
             + [(3, 4), (3, 9), (4, 9)])
    g = csr_from_edges(12, edges)
    g.membership = np.array([0] * 4 + [1] * 4 + [2] * 4, dtype=np.int32)
    return g


def appendix_graph() -> Graph:
    """Graph of the crossover/mutation example (appendix figure): triangles {1,2,3} and
    {6,7,8}, node 4 joined to 1,2,3, node 5 joined to 6,7,8, and the bridge 4-5 (paper ids
    minus one here)."""
    edges = [(0, 1), (1, 2), (2, 0), (3, 0), (3, 1), (3, 2),
             (5, 6), (6, 7), (7, 5), (4, 5), (4, 6), (4, 7), (3, 4)]
    g = csr_from_edges(8, edges)
    g.membership = np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.int32)
    return g


def two_cliques(a: int, b: int) -> Graph:
    """K_a and K_b joined by one bridge between node 0 and node a."""
    edges = _clique(list(range(a))) + _clique(list(range(a, a + b))) + [(0, a)]
    g = csr_from_edges(a + b, edges)
    g.membership = np.array([0] * a + [1] * b, dtype=np.int32)
    return g


def star(n: int) -> Graph:
    return csr_from_edges(n, [(0, i) for i in range(1, n)])


def path(n: int) -> Graph:
    return csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])


def complete(n: int) -> Graph:
    return csr_from_edges(n, _clique(list(range(n))))


def with_isolated(g: Graph, extra: int, seed: int = 0) -> Graph:
    """g plus `extra` isolated nodes, all ids shuffled."""
    n = g.n + extra
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    edges = np.stack([perm[src], perm[g.col]], axis=1)
    return csr_from_edges(n, edges)


def gnp(n: int, p: float, seed: int) -> Graph:
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < p
    return csr_from_edges(n, np.stack([iu[0][keep], iu[1][keep]], axis=1))


# ------------------------------------------------------------------------------------------
# LFR-style planted partition
# ------------------------------------------------------------------------------------------
def _powerlaw_sample(rng, tau: float, lo: float, hi: float, size: int) -> np.ndarray:
    """Inverse-CDF samples of the continuous power law p(x) ~ x^-tau on [lo, hi]."""
    u = rng.random(size)
    a = 1.0 - tau
    return (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)


def _powerlaw_mean(tau: float, lo: float, hi: float) -> float:
    a, b = 1.0 - tau, 2.0 - tau
    return (a / b) * (hi ** b - lo ** b) / (hi ** a - lo ** a)


def solve_kmin(tau: float, mean: float, kmax: float) -> float:
    """k_min of a continuous truncated power law on [k_min, kmax] with the given mean."""
    lo, hi = 1e-6, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _powerlaw_mean(tau, mid, kmax) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def planted_partition(n: int, mean_deg: float, max_deg: int, mu: float, cmin: int, cmax: int,
                      tau1: float = 2.5, tau2: float = 1.5, seed: int = 0) -> Graph:
    rng = np.random.default_rng(seed)
    max_deg = min(max_deg, n - 1)
    kmin = solve_kmin(tau1, mean_deg, max_deg)
    deg = np.rint(_powerlaw_sample(rng, tau1, kmin, max_deg, n)).astype(np.int64)
    deg = np.clip(deg, 1, max_deg)

    # community sizes ~ power law (tau2) on [cmin, cmax], summing to n
    cmin = min(cmin, n)
    cmax = max(min(cmax, n), cmin)
    sizes = []
    total = 0
    while total < n:
        s = int(round(float(_powerlaw_sample(rng, tau2, cmin, cmax, 1)[0])))
        s = max(cmin, min(cmax, s))
        sizes.append(s)
        total += s
    sizes[-1] -= total - n
    if sizes[-1] < cmin and len(sizes) > 1:
        rest = sizes.pop()
        for t in rng.integers(0, len(sizes), size=rest):
            sizes[t] += 1
    sizes = np.array(sizes, dtype=np.int64)
    k = len(sizes)

    # random assignment of nodes to communities
    memb = np.repeat(np.arange(k), sizes)
    rng.shuffle(memb)
    csize = sizes[memb]

    k_in = np.minimum(np.rint((1.0 - mu) * deg).astype(np.int64), csize - 1)
    k_in = np.maximum(k_in, 0)
    k_out = deg - k_in

    # intra-community configuration model: shuffle stubs inside each community, pair them
    stub_node = np.repeat(np.arange(n), k_in)
    stub_comm = memb[stub_node]
    order = np.lexsort((rng.random(len(stub_node)), stub_comm))
    stub_node, stub_comm = stub_node[order], stub_comm[order]
    seg_start = np.searchsorted(stub_comm, stub_comm, side="left")
    pos = np.arange(len(stub_node)) - seg_start
    first = (pos % 2 == 0)
    nxt = np.arange(len(stub_node)) + 1
    ok = first & (nxt < len(stub_node))
    ok[ok] &= stub_comm[nxt[ok]] == stub_comm[ok]
    e_in = np.stack([stub_node[ok], stub_node[nxt[ok]]], axis=1)

    # inter-community configuration model over all outgoing stubs
    out_node = np.repeat(np.arange(n), k_out)
    rng.shuffle(out_node)
    if len(out_node) % 2:
        out_node = out_node[:-1]
    e_out = out_node.reshape(-1, 2)
    e_out = e_out[memb[e_out[:, 0]] != memb[e_out[:, 1]]]

    edges = np.concatenate([e_in, e_out])
    perm = rng.permutation(n)           # scatter node ids: communities are not contiguous
    edges = perm[edges]
    g = csr_from_edges(n, edges)
    new_memb = np.empty(n, dtype=np.int32)
    new_memb[perm] = memb
    g.membership = new_memb
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    inter = int(np.count_nonzero(new_memb[src] != new_memb[g.col]))
    g.info = dict(kind="planted_partition", n=n, target_mean_deg=mean_deg, max_deg=max_deg,
                  mu=mu, cmin=cmin, cmax=cmax, tau1=tau1, tau2=tau2, seed=seed, kmin=kmin,
                  m=g.m, mean_deg=float(2 * g.m / n), realised_mu=inter / max(1, 2 * g.m),
                  communities=k, realised_max_deg=int(np.diff(g.row_ptr).max()))
    return g


# ------------------------------------------------------------------------------------------
# Workload recipes (sizes of the paper's synthetic studies, scaled as the benchmark states)
# ------------------------------------------------------------------------------------------
GA_DEFAULT = dict(pop_size=100, generations=100, crossover_p=0.9, mutation_p=0.1,
                  parents_per_child=4, seed=0)


def small_1k(seed: int = 0) -> Graph:
    """|V| = 1,000, mean degree 10, max 50, communities 20-100, mu = 0.3."""
    return planted_partition(1000, 10, 50, 0.3, 20, 100, seed=seed)


def mid_40k(mu: float, seed: int = 0) -> Graph:
    """|V| = 40,000, mean degree 20, max 200, communities 20-1000."""
    return planted_partition(40000, 20, 200, mu, 20, 1000, seed=seed)


def large_1m(seed: int = 0) -> Graph:
    """|V| = 1,000,000, mean degree 15, max 1000, communities 50-5000, mu = 0.4."""
    return planted_partition(1_000_000, 15, 1000, 0.4, 50, 5000, seed=seed)


def batch_params(count: int = 256, seed: int = 0):
    """Per-graph parameters of the batched form: |V| log-uniform in [500, 50000], mean degree
    log-uniform in [5, 30], mu uniform in [0.1, 0.6]; graph seed = index."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(500), math.log(50000)))))
        k = float(math.exp(rng.uniform(math.log(5), math.log(30))))
        mu = float(rng.uniform(0.1, 0.6))
        out.append(dict(n=n, mean_deg=k, mu=mu, seed=i))
    return out


def batch_graph(p: dict) -> Graph:
    n, k = p["n"], p["mean_deg"]
    return planted_partition(n, k, max(int(4 * k), 10), p["mu"], 20, max(100, n // 20),
                             seed=p["seed"])


def request_stream(count: int, rate: float, seed: int = 0):
    """Poisson arrivals (rate per second); |V| log-uniform in [1000, 200000], mean degree
    uniform in [10, 25], mu uniform in [0.1, 0.6]."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1000), math.log(200000)))))
        out.append(dict(arrival=float(t[i]), n=n, mean_deg=float(rng.uniform(10, 25)),
                        mu=float(rng.uniform(0.1, 0.6)), seed=10_000 + i))
    return out
