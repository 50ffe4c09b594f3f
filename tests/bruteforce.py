"""Independent brute-force references used to pin the oracle (tests only).

Nothing here follows the oracle's code path: partitions are enumerated as restricted-growth
strings, objectives come from the adjacency matrix and pair sums rather than from a CSR scan
and a community histogram, and ranks come from repeated extraction of the non-dominated set.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def all_partitions(n: int) -> np.ndarray:
    """Every set partition of n nodes as a restricted-growth string (row), Bell(n) rows."""
    rows = np.zeros((1, 1), dtype=np.int8)
    mx = np.zeros(1, dtype=np.int8)
    for _ in range(1, n):
        reps = (mx + 2).astype(np.int64)
        idx = np.repeat(np.arange(len(rows)), reps)
        nxt = np.concatenate([np.arange(r) for r in reps]).astype(np.int8)
        rows = np.concatenate([rows[idx], nxt[:, None]], axis=1)
        mx = np.maximum(mx[idx], nxt)
    return rows


def adjacency(g) -> np.ndarray:
    Amat = np.zeros((g.n, g.n), dtype=np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    Amat[src, g.col] = 1
    return Amat


def objectives_bruteforce(g, parts: np.ndarray):
    """(A, S) for many partitions at once, from pair sums over the adjacency matrix:
    A = sum_{i,j} A_ij [c_i = c_j], S = sum_{i,j} k_i k_j [c_i = c_j]."""
    Amat = adjacency(g)
    k = Amat.sum(1)
    same = parts[:, :, None] == parts[:, None, :]
    A = np.einsum("pij,ij->p", same.astype(np.int64), Amat)
    S = np.einsum("pij,ij->p", same.astype(np.int64), np.outer(k, k))
    return A, S


def pareto_points(keys):
    """Distinct non-dominated (k1, k2) pairs (minimisation), sorted by k1."""
    pts = sorted(set(map(tuple, keys)))
    front = []
    best2 = None
    for k1, k2 in pts:          # ascending k1, then k2
        if best2 is None or k2 < best2:
            front.append((k1, k2))
            best2 = k2
    return front


def ranks_by_peeling(k1, k2) -> np.ndarray:
    """rank 1 = non-dominated; rank r = non-dominated once ranks < r are removed."""
    n = len(k1)
    rank = np.zeros(n, dtype=np.int32)
    left = set(range(n))
    r = 1
    while left:
        cur = [p for p in left
               if not any(k1[q] <= k1[p] and k2[q] <= k2[p] and (k1[q] < k1[p] or k2[q] < k2[p])
                          for q in left)]
        for p in cur:
            rank[p] = r
        left -= set(cur)
        r += 1
    return rank


def frac_objectives(g, labels):
    """Exact (f1, f2) as fractions from the paper's formula with |E(c)| and community degree
    sums counted over the edge list (each undirected edge once)."""
    m = g.m
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    und = src < g.col
    intra = int(np.count_nonzero(labels[src[und]] == labels[g.col[und]]))
    deg = np.diff(g.row_ptr)
    sums = {}
    for v in range(g.n):
        sums[int(labels[v])] = sums.get(int(labels[v]), 0) + int(deg[v])
    f1 = 1 - Fraction(intra, m)
    f2 = sum((Fraction(s, 2 * m) ** 2 for s in sums.values()), Fraction(0))
    return f1, f2
