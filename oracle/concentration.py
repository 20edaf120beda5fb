"""Concentrations of the connected k-vertex patterns (oracle; test
infrastructure only).

The paper compares its counts with MCMC estimators of the concentration
of a pattern: its count divided by the total count of all connected
patterns of the same size (Sec. 6.3, comparison with MCMC).  The sampler
counts edge-induced copies (embeddings / |Aut|).  Vertex-induced counts
follow from them: every k-vertex set that induces a connected graph G
contains s(H, G) copies of H, where s(H, G) is the number of spanning
subgraphs of G isomorphic to H, so

    copies(H) = sum over G with at least H's edges of s(H, G) induced(G),

an upper-triangular system solved from the densest pattern down.  Here
s(H, G) is counted as the embeddings of H in G (brute force) over |Aut(H)|,
and induced counts are also computed directly on tiny graphs by listing
every k-vertex set, which pins the inversion.
"""

from __future__ import annotations

import itertools
from fractions import Fraction

from .judges import brute_force
from .pattern import automorphisms


class _Tiny:
    """A pattern viewed as a data graph (what brute_force reads)."""

    def __init__(self, k, edges):
        self.n = k
        self._adj = [set() for _ in range(k)]
        for a, b in edges:
            self._adj[a].add(b)
            self._adj[b].add(a)

    def adjacency_sets(self):
        return self._adj


def _canon(k, edges):
    best = None
    for perm in itertools.permutations(range(k)):
        e = tuple(sorted(tuple(sorted((perm[a], perm[b]))) for a, b in edges))
        if best is None or e < best:
            best = e
    return best


def spanning_copies(h, g) -> int:
    """s(H, G): copies of pattern h (k, edges) as a spanning subgraph of the
    same-size pattern g."""
    kh, eh = h
    kg, eg = g
    assert kh == kg
    return brute_force(_Tiny(kg, eg), kh, eh) // automorphisms(kh, eh)


def induced_from_copies(patterns, copies):
    """Vertex-induced counts from edge-induced copy counts (exact rationals
    when the copies are integers or Fractions)."""
    n = len(patterns)
    s = [[spanning_copies(patterns[h], patterns[g]) if len(patterns[g][1]) >= len(patterns[h][1]) else 0
          for g in range(n)] for h in range(n)]
    order = sorted(range(n), key=lambda i: -len(patterns[i][1]))
    ind = [None] * n
    for h in order:
        v = Fraction(copies[h]) if not isinstance(copies[h], float) else copies[h]
        for g in range(n):
            if g != h and s[h][g]:
                v -= s[h][g] * ind[g]
        ind[h] = v / s[h][h]
    return ind


def induced_direct(g, patterns):
    """Vertex-induced counts on a tiny data graph by listing every k-set."""
    k = patterns[0][0]
    index = {_canon(kk, e): i for i, (kk, e) in enumerate(patterns)}
    adj = g.adjacency_sets()
    out = [0] * len(patterns)
    for vs in itertools.combinations(range(g.n), k):
        e = [(a, b) for a, b in itertools.combinations(range(k), 2) if vs[b] in adj[vs[a]]]
        c = _canon(k, e)
        if c in index:
            out[index[c]] += 1
    return out


def normalise(values):
    tot = sum(values)
    return [v / tot if tot else 0 for v in values]


def variation_distance(p, q) -> float:
    return 0.5 * sum(abs(float(a) - float(b)) for a, b in zip(p, q))
