"""Graph-object adapters: networkx, igraph, scipy.sparse and plain edge lists to the symmetric
int32 CSR that ``Graph`` / ``hpmocd_graph_create`` take, and labels back to communities of
the original node keys.

Section 2.1's graph is simple, undirected and unweighted, so conversion symmetrises directed
input, drops weights, and either drops self-loops and repeated edges (the default) or lets
the library reject them (``strict=True``). Node v of the CSR is the v-th node in the source
object's own node order; ``Converted.nodes`` maps back.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Converted:
    row_ptr: np.ndarray   # int32 [n + 1]
    col: np.ndarray       # int32 [2m], each adjacency list ascending
    nodes: list           # CSR index -> original node key

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1


def _csr(n: int, src, dst, strict: bool):
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.shape != dst.shape:
        raise ValueError("edge endpoint arrays differ in length")
    if src.size and (min(src.min(), dst.min()) < 0 or max(src.max(), dst.max()) >= n):
        raise ValueError("edge endpoint outside [0, n)")
    if not strict:
        keep = src != dst
        lo = np.minimum(src[keep], dst[keep])
        hi = np.maximum(src[keep], dst[keep])
        key = np.unique(lo * n + hi)
        lo, hi = key // n, key % n
        a = np.concatenate([lo, hi])
        b = np.concatenate([hi, lo])
    else:  # both directions of every listed edge, kept as given (the library validates)
        a = np.concatenate([src, dst])
        b = np.concatenate([dst, src])
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, a + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    if row_ptr[-1] >= 2**31:
        raise ValueError("too many arcs for int32 CSR")
    return row_ptr.astype(np.int32), b.astype(np.int32)


def from_edges(n: int, edges, strict: bool = False, nodes=None) -> Converted:
    """Edge list of (u, v) pairs over nodes 0..n-1 (either orientation, any order)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col = _csr(n, e[:, 0], e[:, 1], strict)
    return Converted(rp, col, list(range(n)) if nodes is None else list(nodes))


def from_networkx(G, strict: bool = False) -> Converted:
    """networkx Graph / DiGraph / MultiGraph (duck-typed: ``nodes`` and ``edges()``)."""
    nodes = list(G.nodes())
    index = {v: i for i, v in enumerate(nodes)}
    pairs = [(index[u], index[v]) for u, v in G.edges()]
    return from_edges(len(nodes), pairs if pairs else np.zeros((0, 2)), strict, nodes)


def from_igraph(g, strict: bool = False) -> Converted:
    """python-igraph Graph (duck-typed: ``vcount()`` and ``get_edgelist()``); vertex ids are
    already 0..n-1, and ``vs['name']`` (when present) names the nodes."""
    n = g.vcount()
    try:
        names = list(g.vs["name"])
    except Exception:
        names = list(range(n))
    el = g.get_edgelist()
    return from_edges(n, el if el else np.zeros((0, 2)), strict, names)


def from_scipy(A, strict: bool = False) -> Converted:
    """Square scipy.sparse adjacency matrix; nonzero (i, j) or (j, i) is an edge."""
    A = A.tocoo()
    if A.shape[0] != A.shape[1]:
        raise ValueError("adjacency matrix must be square")
    nz = A.data != 0
    rp, col = _csr(A.shape[0], A.row[nz], A.col[nz], strict)
    return Converted(rp, col, list(range(A.shape[0])))


def communities(labels, nodes=None) -> list:
    """One row of front labels -> list of sets of node keys, largest first."""
    labels = np.asarray(labels)
    keys = list(range(len(labels))) if nodes is None else nodes
    groups: dict = {}
    for i, c in enumerate(labels.tolist()):
        groups.setdefault(c, set()).add(keys[i])
    return sorted(groups.values(), key=len, reverse=True)


def detect(G, *, stream=None, **params):
    """Converts a graph object, runs Alg. 1 on the device and returns (front, communities of
    the selected solution, Converted). params: pop_size, generations, crossover_p,
    mutation_p, parents_per_child, seed."""
    from . import Graph, run
    if hasattr(G, "get_edgelist"):
        conv = from_igraph(G)
    elif hasattr(G, "tocoo"):
        conv = from_scipy(G)
    else:
        conv = from_networkx(G)
    front = run(Graph(conv.row_ptr, conv.col), stream=stream, **params)
    return front, communities(front.labels[front.selected], conv.nodes), conv
