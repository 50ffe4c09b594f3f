"""Graph-object adapters to CSR (host only): networkx (installed), an igraph-shaped object
(python-igraph is not installed here, so only its interface is exercised), scipy.sparse and
edge lists; every conversion gives the symmetric sorted CSR the library validates."""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2506_01752_amd as hp
from paper_2506_01752_amd import adapters as ad
import synth


def csr_equal(conv, g):
    return np.array_equal(conv.row_ptr, g.row_ptr) and np.array_equal(conv.col, g.col)


def passes_validation(conv):
    # 0 with a GPU, ERR_HIP (-9) without one: either way validation accepted the CSR
    return hp.graph_create_status(conv.n, conv.row_ptr, conv.col) in (0, -9)


def test_networkx_karate_club():
    G = nx.karate_club_graph()
    conv = ad.from_networkx(G)
    assert conv.n == 34 and len(conv.col) == 2 * G.number_of_edges()
    ref = synth.csr_from_edges(34, list(G.edges()))
    assert csr_equal(conv, ref)
    assert passes_validation(conv)


def test_networkx_keys_directed_multi_and_loops():
    G = nx.MultiDiGraph()
    G.add_edges_from([("a", "b"), ("b", "a"), ("a", "b"), ("b", "c"), ("c", "c"), ("d", "a")])
    G.add_node("e")  # isolated
    conv = ad.from_networkx(G)
    assert conv.nodes == ["a", "b", "c", "d", "e"]
    ref = synth.csr_from_edges(5, [(0, 1), (1, 2), (3, 0)])
    assert csr_equal(conv, ref)
    assert passes_validation(conv)
    # strict keeps self-loops and repeats for the library to reject
    strict = ad.from_networkx(G, strict=True)
    assert hp.graph_create_status(strict.n, strict.row_ptr, strict.col) in (-3, -4)


class FakeIgraph:
    def __init__(self, n, edges, names=None):
        self._n, self._e = n, edges
        self.vs = {"name": names} if names is not None else {}

    def vcount(self):
        return self._n

    def get_edgelist(self):
        return list(self._e)


def test_igraph_shaped_object():
    edges = [(0, 1), (1, 2), (2, 0), (2, 3)]
    conv = ad.from_igraph(FakeIgraph(4, edges, names=["w", "x", "y", "z"]))
    assert conv.nodes == ["w", "x", "y", "z"]
    assert csr_equal(conv, synth.csr_from_edges(4, edges))
    conv = ad.from_igraph(FakeIgraph(4, edges))
    assert conv.nodes == [0, 1, 2, 3]


def test_scipy_sparse_upper_or_full():
    g = synth.fig1_graph()
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    upper = src < g.col
    A = sp.coo_matrix((np.ones(upper.sum()), (src[upper], g.col[upper])), shape=(n, n)).tocsr()
    assert csr_equal(ad.from_scipy(A), g)
    assert csr_equal(ad.from_scipy(A + A.T), g)
    with pytest.raises(ValueError):
        ad.from_scipy(sp.coo_matrix((2, 3)))


def test_edge_list_errors_and_communities():
    with pytest.raises(ValueError):
        ad.from_edges(3, [(0, 3)])
    labels = np.array([5, 5, 2, 5, 2])
    com = ad.communities(labels, nodes=list("abcde"))
    assert com == [{"a", "b", "d"}, {"c", "e"}]
