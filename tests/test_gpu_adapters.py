"""detect() on graph objects (section 4's graph input, converted to the CSR of section 2.1):
its front equals the CPU oracle's run on the converted CSR, bit for bit, and its communities
are the selected solution's label classes named by the original node keys."""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_01752_amd as m
    m.lib()
    return m


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def _check_against_oracle(front, coms, conv, kw):
    ref = oracle.run(conv.row_ptr, conv.col, **kw)
    assert front.labels.shape == ref.labels.shape
    assert np.array_equal(front.labels, ref.labels)
    assert np.array_equal(front.A, ref.A) and np.array_equal(front.S, ref.S)
    assert np.array_equal(bits(front.f1), bits(ref.f1))
    assert np.array_equal(bits(front.f2), bits(ref.f2))
    assert front.selected == ref.selected
    # the communities are the label classes of the selected row, in node keys
    sel = front.labels[front.selected]
    want = {}
    for i, c in enumerate(sel.tolist()):
        want.setdefault(c, set()).add(conv.nodes[i])
    assert sorted(map(sorted, coms)) == sorted(map(sorted, want.values()))
    assert sum(len(c) for c in coms) == conv.n


def test_detect_networkx_equals_oracle(hp):
    import torch
    from paper_2506_01752_amd import adapters as ad
    G = nx.relabel_nodes(nx.karate_club_graph(), {i: f"m{i}" for i in range(34)})
    s = torch.cuda.Stream()
    kw = dict(pop_size=40, generations=30, crossover_p=0.9, mutation_p=0.1,
              parents_per_child=4, seed=7)
    front, coms, conv = ad.detect(G, stream=s, **kw)
    _check_against_oracle(front, coms, conv, kw)
    assert sorted(set().union(*coms)) == sorted(G.nodes())
    # and the same run from the CSR entry point
    ref = hp.run(hp.Graph(conv.row_ptr, conv.col), stream=s, **kw)
    assert np.array_equal(front.labels, ref.labels) and front.selected == ref.selected
    print("communities:", [len(c) for c in coms], flush=True)


def test_detect_directed_multigraph_and_scipy_equal_oracle(hp):
    import torch
    from paper_2506_01752_amd import adapters as ad
    s = torch.cuda.Stream()
    kw = dict(pop_size=24, generations=12, crossover_p=0.8, mutation_p=0.2,
              parents_per_child=3, seed=11)
    # a directed multigraph with repeated arcs, both orientations and a self-loop:
    # symmetrised and deduplicated to a simple graph
    D = nx.MultiDiGraph()
    rng = np.random.default_rng(4)
    keys = [f"n{k:03d}" for k in rng.permutation(300)]
    D.add_nodes_from(keys)
    for _ in range(1500):
        u, v = rng.integers(0, 300, size=2)
        D.add_edge(keys[u], keys[v])
    D.add_edge(keys[0], keys[0])
    front, coms, conv = ad.detect(D, stream=s, **kw)
    _check_against_oracle(front, coms, conv, kw)
    # a scipy.sparse adjacency matrix (weights ignored, one triangle only given)
    A = sp.random(500, 500, density=0.01, random_state=5, format="coo")
    A = sp.triu(A, k=1).tocoo()
    A.data[:] = rng.uniform(0.5, 3.0, size=A.nnz)
    front, coms, conv = ad.detect(A, stream=s, **kw)
    _check_against_oracle(front, coms, conv, kw)
