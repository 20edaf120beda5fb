"""Oracle pattern compiler -- TEST INFRASTRUCTURE ONLY.

Plain Python restatement of the pattern-side analysis of the paper:
  * the remaining pattern P_i and its hop groups (Sec. 4.2.2, Eq. Pi);
  * the auxiliary arrays A^pi: |B|, |F1|, |I1|, |I_effective|, |F2|
    (Sec. 4.2.3, Definition "Auxiliary Arrays");
  * the decision function D^pi with its certainty value
    (Sec. 5.1, Definition "Decision Function");
  * the greedy matching order (Sec. 5.2, Algorithm 2 "Matching Order
    Construction").

Readings taken where the paper is open (each listed in the design notes):
  * E^{>=2hop} is taken over E_P, exactly as written in the definition;
  * the threshold comparison is exact (rational arithmetic, beta = 4/5);
  * Algorithm 2 breaks score ties by the smallest pattern-vertex id and
    scores |F1| + |I1| (the full I1, as written);
  * |F2| counts edges between hop-1 and hop-2 vertices (not vertices).
"""

from __future__ import annotations

import itertools
from fractions import Fraction

MODES = ("uniform", "switch", "always", "learned")


def _adj(k, edges):
    adj = [set() for _ in range(k)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    return adj


def _bfs(adj, allowed, src):
    dist = {src: 0}
    frontier = [src]
    while frontier:
        nxt = []
        for a in frontier:
            for b in sorted(adj[a]):
                if b in allowed and b not in dist:
                    dist[b] = dist[a] + 1
                    nxt.append(b)
        frontier = nxt
    return dist


def _components(vertices, edges):
    parent = {v: v for v in vertices}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    comps = len(vertices)
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
            comps -= 1
    return comps


def step_analysis(k, edges, order, i):
    """Analysis of step i (0-based) of matching order ``order``.

    Returns a dict with b, f1, i1 (= |I1|), ie (= |I_effective|), f2 and the
    certainty value, for the pattern vertex u_i = order[i].
    """
    adj = _adj(k, edges)
    u = order[i]
    prefix = set(order[:i])
    remaining = set(order[i:])
    b = sum(1 for w in adj[u] if w in prefix)
    dist = _bfs(adj, remaining, u)
    h1 = {w for w, d in dist.items() if d == 1}
    h2 = {w for w, d in dist.items() if d == 2}
    e_i = [(a, c) for a, c in edges if a in remaining and c in remaining]
    i1 = [(a, c) for a, c in e_i if a in h1 and c in h1]
    v_ind = {a for e in i1 for a in e}
    ie = len(v_ind) - _components(v_ind, i1) if v_ind else 0
    f2 = sum(1 for a, c in e_i if (a in h1 and c in h2) or (a in h2 and c in h1))
    v_ge2 = {w for w, d in dist.items() if d >= 2}
    e_ge2 = [(a, c) for a, c in edges if a in v_ge2 or c in v_ge2]
    certainty = 1 - Fraction(len(e_ge2) - len(v_ge2), len(remaining))
    return {"u": u, "b": b, "f1": len(h1), "i1": len(i1), "ie": ie, "f2": f2, "certainty": certainty}


def matching_order(k, edges):
    """Algorithm 2: greedy order maximising |F1| + |I1| over the frontier."""
    adj = _adj(k, edges)
    order = []
    for i in range(k):
        if i == 0:
            cands = list(range(k))
        else:
            cands = sorted({w for x in order for w in adj[x] if w not in order})
        best, best_s = None, None
        for u in cands:
            a = step_analysis(k, edges, order + [u] + [w for w in range(k) if w not in order and w != u], i)
            s = a["f1"] + a["i1"]
            if best_s is None or s > best_s:
                best, best_s = u, s
        order.append(best)
    return order


def automorphisms(k, edges):
    es = {(min(a, b), max(a, b)) for a, b in edges}
    cnt = 0
    for perm in itertools.permutations(range(k)):
        if all((min(perm[a], perm[b]), max(perm[a], perm[b])) in es for a, b in es):
            cnt += 1
    return cnt


def is_connected(k, edges):
    if k == 0:
        return False
    return len(_bfs(_adj(k, edges), set(range(k)), 0)) == k


def check_order(k, edges, order):
    """Every prefix of the order must induce a connected subpattern."""
    if sorted(order) != list(range(k)):
        raise ValueError("order is not a permutation of the pattern vertices")
    adj = _adj(k, edges)
    for i in range(1, k):
        if not any(w in order[:i] for w in adj[order[i]]):
            raise ValueError(f"order position {i} has no matched neighbour")


def compile_pattern(k, edges, order=None, mode="switch", beta=Fraction(4, 5)):
    """Compile a pattern for the sampler.

    mode: 'uniform' (D = 0 everywhere), 'switch' (the decision function with
    threshold beta), 'always' (D = 1 everywhere), 'learned' (same decisions
    as 'switch'; weighted steps read learned tables).  ``beta`` may be a
    Fraction, or float('inf') / float('-inf') for the sweep extremes.
    """
    if mode not in MODES:
        raise ValueError(f"unknown mode {mode}")
    edges = [(min(a, b), max(a, b)) for a, b in edges]
    if not (2 <= k <= 8):
        raise ValueError("pattern size must be in [2, 8]")
    if not is_connected(k, edges):
        raise ValueError("pattern is not connected")
    if order is None:
        order = matching_order(k, edges)
    order = list(order)
    check_order(k, edges, order)
    pos = {u: i for i, u in enumerate(order)}
    adj = _adj(k, edges)
    steps = []
    for i in range(k):
        a = step_analysis(k, edges, order, i)
        bmask = 0
        for w in adj[order[i]]:
            if pos[w] < i:
                bmask |= 1 << pos[w]
        if mode == "uniform":
            d = 0
        elif mode == "always":
            d = 1
        else:
            d = 1 if a["certainty"] >= beta else 0
        a["bmask"] = bmask
        a["decision"] = d
        steps.append(a)
    return {"k": k, "order": order, "steps": steps, "aut": automorphisms(k, edges), "mode": mode}
