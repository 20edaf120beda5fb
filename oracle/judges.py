"""Exact embedding counts -- TEST INFRASTRUCTURE ONLY.

C(G, P) is the number of injective maps M: V_P -> V_G that send every
pattern edge to a graph edge (Sec. 2.1).  It counts labelled embeddings, so
the number of distinct subgraph copies is C / |Aut(P)|.

  * ``brute_force``: the definition written out over all injective maps
    (tiny graphs only);
  * ``backtrack``: the same count by backtracking over a connected order
    (C code in the oracle library);
  * closed forms for special shapes, each checked against the brute force
    in the tests before it is trusted on larger graphs.
"""

from __future__ import annotations

import ctypes
import itertools
import math

import numpy as np

from . import lib, _p
from .pattern import matching_order


def brute_force(g, k, edges) -> int:
    adj = g.adjacency_sets()
    cnt = 0
    for m in itertools.permutations(range(g.n), k):
        if all(m[b] in adj[m[a]] for a, b in edges):
            cnt += 1
    return cnt


def backtrack(g, k, edges, order=None) -> int:
    if order is None:
        order = matching_order(k, edges)
    adjm = np.zeros(8, dtype=np.uint8)
    for a, b in edges:
        adjm[a] |= 1 << b
        adjm[b] |= 1 << a
    ordm = np.zeros(8, dtype=np.uint8)
    ordm[:k] = order
    off = np.ascontiguousarray(g.off, dtype=np.uint64)
    nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
    return int(lib().orc_count_embeddings(_p(off), _p(nbr), g.n, g.nnz, _p(adjm), _p(ordm), k))


def rooted_counts(g, k, edges, order) -> np.ndarray:
    """n_(v): embeddings with pattern vertex order[0] mapped to v, per v."""
    adjm = np.zeros(8, dtype=np.uint8)
    for a, b in edges:
        adjm[a] |= 1 << b
        adjm[b] |= 1 << a
    ordm = np.zeros(8, dtype=np.uint8)
    ordm[:k] = order
    off = np.ascontiguousarray(g.off, dtype=np.uint64)
    nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
    out = np.zeros(max(g.n, 1), dtype=np.uint64)
    lib().orc_rooted_counts(_p(off), _p(nbr), g.n, g.nnz, _p(adjm), _p(ordm), k, _p(out))
    return out[: g.n]


def clique_embeddings(g, k, threads: int = 1) -> int:
    """threads != 1: the vertices spread over host threads (0 = all)."""
    off = np.ascontiguousarray(g.off, dtype=np.uint64)
    nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
    if threads != 1:
        copies = int(lib().orc_count_cliques_parallel(_p(off), _p(nbr), g.n, g.nnz, k, threads))
    else:
        copies = int(lib().orc_count_cliques(_p(off), _p(nbr), g.n, g.nnz, k))
    return copies * math.factorial(k)


def _adjacency(g):
    import scipy.sparse as sp
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.off).astype(np.int64))
    return sp.csr_matrix((np.ones(g.nnz, dtype=np.float64), (rows, g.nbr.astype(np.int64))), shape=(g.n, g.n))


def triangle_embeddings(g) -> int:
    """trace(A^3) = 6 * #triangles = number of triangle embeddings."""
    A = _adjacency(g)
    return int(round((A @ A).multiply(A).sum()))


def four_cycle_embeddings(g) -> int:
    """Each 4-cycle has two diagonals {u, w}; with c(u, w) common neighbours a
    diagonal closes C(c, 2) cycles, so copies = sum_{u<w} C(c, 2) / 2 and
    embeddings = 8 * copies = 2 * sum_{u != w} C(c(u, w), 2)."""
    A = _adjacency(g)
    A2 = (A @ A).tocoo()
    off_diag = A2.row != A2.col
    c = A2.data[off_diag].astype(np.int64)
    return int(2 * np.sum(c * (c - 1) // 2))


def star_embeddings(g, leaves) -> int:
    """k! * sum_v C(d(v), k): centre at v, leaves an ordered k-subset of N(v)."""
    d = g.degrees()
    return int(sum(math.perm(int(x), leaves) for x in d if x >= leaves))


def wedge_embeddings(g) -> int:
    d = g.degrees()
    return int(np.sum(d * (d - 1)))
