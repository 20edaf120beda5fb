"""Pins of the oracle's pattern compiler (Algorithm 2, auxiliary arrays,
decision function)."""

import itertools
from fractions import Fraction

import pytest

import synth
from oracle import judges
from oracle.pattern import compile_pattern, step_analysis, automorphisms, matching_order, check_order
from conftest import golden_path


def _golden_rows():
    rows = []
    for line in open(golden_path("pattern_signatures.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, aut, order, dec, steps = [x.strip() for x in line.split("|")]
        rows.append((name, int(aut), [int(x) for x in order.split()], dec,
                     [tuple(int(y) for y in s.split(",")) for s in steps.split()]))
    return rows


@pytest.mark.parametrize("name,aut,order,dec,steps", _golden_rows())
def test_signature_golden(name, aut, order, dec, steps):
    p = synth.named_pattern(name)
    c = compile_pattern(p.k, p.edges)
    assert c["aut"] == aut
    assert c["order"] == order
    assert "".join("A" if s["decision"] else "U" for s in c["steps"]) == dec
    assert [(s["b"], s["f1"], s["i1"], s["ie"], s["f2"]) for s in c["steps"]] == steps


def test_house_has_one_uniform_step_of_five():
    p = synth.named_pattern("house")
    c = compile_pattern(p.k, p.edges)
    assert sum(1 - s["decision"] for s in c["steps"]) == 1


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7, 8])
def test_cliques_have_certainty_one(k):
    p = synth.patterns.clique(k)
    c = compile_pattern(p.k, p.edges)
    assert all(s["certainty"] == 1 for s in c["steps"])


def test_certainty_at_most_one_every_order():
    # |E^{>=2hop}| >= |V^{>=2hop}| because every vertex at distance >= 2 has
    # its own edge towards its BFS parent; so certainty <= 1 (as the
    # definition of the decision function states).
    pats = [p for p, _ in synth.random_pattern_set(12, seed=4, kmin=4, kmax=6)]
    for p in pats:
        adj = p.adj
        for order in itertools.permutations(range(p.k)):
            ok = all(any(adj[order[i]] >> order[j] & 1 for j in range(i)) for i in range(1, p.k))
            if not ok:
                continue
            for i in range(p.k):
                assert step_analysis(p.k, p.edges, list(order), i)["certainty"] <= 1


def test_matching_order_prefixes_connected():
    for p, _ in synth.random_pattern_set(32, seed=3):
        order = matching_order(p.k, p.edges)
        check_order(p.k, p.edges, order)


def test_b_plus_f1_is_pattern_degree():
    # Every neighbour of u_i is either matched earlier (B) or in hop 1 of P_i.
    for p, _ in synth.random_pattern_set(20, seed=5):
        c = compile_pattern(p.k, p.edges)
        deg = [bin(a).count("1") for a in p.adj]
        for s in c["steps"]:
            assert s["b"] + s["f1"] == deg[s["u"]]


def test_first_step_is_alg2_argmax():
    # Algorithm 2 at i = 1 scores every vertex by deg(u) + |edges among N(u)|.
    for p, _ in synth.random_pattern_set(20, seed=6):
        adj = p.adj
        score = []
        for u in range(p.k):
            nb = [w for w in range(p.k) if adj[u] >> w & 1]
            tri = sum(1 for a, b in itertools.combinations(nb, 2) if adj[a] >> b & 1)
            score.append(len(nb) + tri)
        best = max(score)
        assert matching_order(p.k, p.edges)[0] == score.index(best)


def test_automorphism_counts_match_brute_force_on_pattern_itself():
    # |Aut(P)| equals the number of embeddings of P into a graph that is a
    # copy of P, divided by its number of copies there (one).
    for name in ["triangle", "4-cycle", "house", "4-star", "diamond", "5-cycle"]:
        p = synth.named_pattern(name)
        g = synth.csr_from_edges(p.k, [a for a, _ in p.edges], [b for _, b in p.edges])
        assert judges.brute_force(g, p.k, p.edges) == automorphisms(p.k, p.edges)


def test_worked_example_pattern_side():
    fx = _worked_example()
    k = fx["pattern_vertices"]
    edges = fx["pattern_edges"]
    a = step_analysis(k, edges, list(range(k)), fx["step"])
    assert (a["b"], a["f1"], a["ie"], a["f2"]) == (fx["expect_b"], fx["expect_f1"], fx["expect_ie"], fx["expect_f2"])


def _worked_example():
    fx = {}
    for line in open(golden_path("worked_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key.endswith("edges"):
            fx[key] = [tuple(int(x) for x in v.split("-")) for v in vals]
        elif key.startswith("expect_T"):
            fx[key] = Fraction(vals[0])
        else:
            fx[key] = int(vals[0])
    return fx


def test_compile_rejects_bad_inputs():
    with pytest.raises(ValueError):
        compile_pattern(4, [(0, 1), (2, 3)])  # disconnected
    with pytest.raises(ValueError):
        compile_pattern(1, [])
    with pytest.raises(ValueError):
        compile_pattern(4, [(0, 1), (1, 2), (2, 3)], order=[0, 2, 1, 3])  # prefix {0,2} disconnected
    with pytest.raises(ValueError):
        compile_pattern(3, [(0, 1), (1, 2), (0, 2)], mode="bogus")


def test_mode_overrides():
    p = synth.named_pattern("4-cycle")
    assert all(s["decision"] == 0 for s in compile_pattern(p.k, p.edges, mode="uniform")["steps"])
    assert all(s["decision"] == 1 for s in compile_pattern(p.k, p.edges, mode="always")["steps"])
    assert all(s["decision"] == 0 for s in compile_pattern(p.k, p.edges, beta=float("inf"))["steps"])


# ------------------------------------------------------------ concentrations

@pytest.mark.parametrize("k", [3, 4, 5])
def test_induced_counts_by_inversion_match_direct_listing(k):
    """Edge-induced copies (brute force) inverted through s(H, G) give the
    vertex-induced counts found by listing every k-vertex set."""
    from oracle import concentration as conc
    pats = [(p.k, list(p.edges)) for p in synth.patterns.connected_patterns(k)]
    for seed in range(3):
        g = synth.graphs.tiny_graph(8, 0.45, 30 + seed)
        copies = [judges.brute_force(g, kk, e) // automorphisms(kk, e) for kk, e in pats]
        inv = conc.induced_from_copies(pats, copies)
        direct = conc.induced_direct(g, pats)
        assert [int(x) for x in inv] == direct and all(x.denominator == 1 for x in inv)


def test_concentrations_on_complete_graph():
    from oracle import concentration as conc
    pats = [(p.k, list(p.edges)) for p in synth.patterns.connected_patterns(4)]
    g = synth.complete_graph(6)
    copies = [judges.brute_force(g, kk, e) // automorphisms(kk, e) for kk, e in pats]
    ind = conc.induced_from_copies(pats, copies)
    # every 4-set of K6 induces K4: C(6, 4) = 15 of them, nothing else
    assert ind[-1] == 15 and all(x == 0 for x in ind[:-1])
    assert conc.normalise(ind)[-1] == 1
    # spanning copies of the 4-path in K4: 4!/2 = 12
    path4 = next(i for i, (kk, e) in enumerate(pats) if len(e) == 3 and max(
        sum(1 for ed in e if v in ed) for v in range(4)) == 2)
    assert conc.spanning_copies(pats[path4], pats[-1]) == 12
