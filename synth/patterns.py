"""Pattern graphs: named shapes and a seeded random pattern set.

A pattern is a small connected undirected graph on vertices ``0..k-1``
(2 <= k <= 8), stored as an edge list and as per-vertex adjacency bitmasks
(``adj[u]`` has bit ``w`` set iff {u, w} is an edge).

The paper names its evaluation patterns but its pattern figure is not
available, so the shapes here are the conventional ones: a k-star is a
centre joined to k leaves (Sec. 2.2), the house is a 4-cycle with an apex
on one of its edges, and the chordal 7-cycle is C7 plus the chord {0, 3}.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass(frozen=True)
class Pattern:
    k: int
    edges: tuple  # tuple of (a, b) with a < b
    name: str = ""

    def __post_init__(self):
        if not (1 <= self.k <= 8):
            raise ValueError("pattern size must be between 1 and 8")
        for a, b in self.edges:
            if not (0 <= a < self.k and 0 <= b < self.k) or a == b:
                raise ValueError(f"bad pattern edge {(a, b)}")

    @property
    def adj(self) -> list:
        m = [0] * self.k
        for a, b in self.edges:
            m[a] |= 1 << b
            m[b] |= 1 << a
        return m

    def adj8(self) -> list:
        """Adjacency bitmasks padded to 8 entries (the C-ABI layout)."""
        return self.adj + [0] * (8 - self.k)

    def is_connected(self) -> bool:
        adj = self.adj
        seen = 1
        frontier = 1
        while frontier:
            nxt = 0
            for u in range(self.k):
                if frontier >> u & 1:
                    nxt |= adj[u]
            frontier = nxt & ~seen
            seen |= nxt
        return seen == (1 << self.k) - 1


def _mk(k, edges, name):
    return Pattern(k=k, edges=tuple(sorted((min(a, b), max(a, b)) for a, b in edges)), name=name)


def clique(k):
    return _mk(k, list(itertools.combinations(range(k), 2)), f"{k}-clique")


def cycle(k):
    return _mk(k, [(i, (i + 1) % k) for i in range(k)], f"{k}-cycle")


def path(k):
    return _mk(k, [(i, i + 1) for i in range(k - 1)], f"{k}-path")


def star(leaves):
    return _mk(leaves + 1, [(0, i) for i in range(1, leaves + 1)], f"{leaves}-star")


NAMED_PATTERNS = {
    "edge": _mk(2, [(0, 1)], "edge"),
    "wedge": path(3),
    "triangle": _mk(3, [(0, 1), (1, 2), (0, 2)], "triangle"),
    "4-cycle": cycle(4),
    "4-clique": clique(4),
    "4-path": path(4),
    "3-star": star(3),
    "diamond": _mk(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)], "diamond"),
    "tailed-triangle": _mk(4, [(0, 1), (1, 2), (0, 2), (2, 3)], "tailed-triangle"),
    "5-clique": clique(5),
    "5-cycle": cycle(5),
    "house": _mk(5, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (1, 4)], "house"),
    "4-star": star(4),
    "6-clique": clique(6),
    "6-cycle": cycle(6),
    "chordal-7-cycle": _mk(7, [(i, (i + 1) % 7) for i in range(7)] + [(0, 3)], "chordal-7-cycle"),
}


def named_pattern(name: str) -> Pattern:
    return NAMED_PATTERNS[name]


def _canonical(k: int, edges) -> tuple:
    best = None
    for perm in itertools.permutations(range(k)):
        e = tuple(sorted((min(perm[a], perm[b]), max(perm[a], perm[b])) for a, b in edges))
        if best is None or e < best:
            best = e
    return best


def random_pattern_set(count: int = 32, seed: int = 3, kmin: int = 4, kmax: int = 7,
                       budget_lo: float = 1e6, budget_hi: float = 1e9):
    """``count`` pairwise non-isomorphic connected patterns with sample budgets.

    Recipe: k uniform in [kmin, kmax]; a uniformly random labelled tree from
    a random Pruefer sequence; every remaining vertex pair becomes an edge
    with probability 1/3; a pattern isomorphic to an earlier one is redrawn.
    Budgets are log-uniform in [budget_lo, budget_hi], rounded to integers.
    Returns a list of (Pattern, budget).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    seen = set()
    out = []
    lo, hi = np.log10(budget_lo), np.log10(budget_hi)
    while len(out) < count:
        k = int(rng.integers(kmin, kmax + 1))
        prufer = [int(x) for x in rng.integers(0, k, size=k - 2)]
        degree = [1] * k
        for x in prufer:
            degree[x] += 1
        edges = []
        for x in prufer:
            leaf = min(i for i in range(k) if degree[i] == 1)
            edges.append((leaf, x))
            degree[leaf] -= 1
            degree[x] -= 1
        rest = [i for i in range(k) if degree[i] == 1]
        edges.append((rest[0], rest[1]))
        have = {(min(a, b), max(a, b)) for a, b in edges}
        for a, b in itertools.combinations(range(k), 2):
            if (a, b) not in have and rng.random() < 1.0 / 3.0:
                have.add((a, b))
        canon = (k, _canonical(k, have))
        if canon in seen:
            continue
        seen.add(canon)
        budget = int(round(10 ** (lo + (hi - lo) * rng.random())))
        out.append((_mk(k, have, f"rand{len(out):02d}_k{k}"), budget))
    return out


def connected_patterns(k: int):
    """Every connected graph on k vertices (2 <= k <= 6) up to isomorphism,
    one representative each, ordered by edge count and then by canonical
    code: 1, 2, 6, 21 and 112 patterns for k = 2..6."""
    if not (2 <= k <= 6):
        raise ValueError("connected_patterns supports 2 <= k <= 6")
    pairs = list(itertools.combinations(range(k), 2))
    seen = {}
    for mask in range(1 << len(pairs)):
        edges = {pairs[j] for j in range(len(pairs)) if mask >> j & 1}
        if len(edges) < k - 1:
            continue
        p = _mk(k, edges, "")
        if not p.is_connected():
            continue
        code = _canonical(k, edges)
        if code not in seen:
            seen[code] = edges
    out = []
    for code in sorted(seen, key=lambda c: (len(seen[c]), c)):
        out.append(_mk(k, seen[code], f"k{k}_{len(out):02d}"))
    return out

