"""Pins of the oracle's tables, sampler and estimator against the paper's
theorems, worked examples and closed forms."""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import judges
from oracle.estimator import eps_hat, direct_stats, run_to_eps, z_value
from oracle.pattern import compile_pattern
from oracle.tree import enumerate_tree
from test_oracle_pattern import _worked_example

MODES = ["uniform", "switch", "always"]


# ------------------------------------------------------------ judges

SMALL_GRAPHS = [synth.graphs.tiny_graph(8, 0.5, s) for s in range(3)] + \
    [synth.graphs.skewed_tiny_graph(9, seed=s) for s in range(2)]


@pytest.mark.parametrize("gi", range(len(SMALL_GRAPHS)))
def test_closed_forms_match_brute_force(gi):
    g = SMALL_GRAPHS[gi]
    P = synth.named_pattern
    assert judges.triangle_embeddings(g) == judges.brute_force(g, 3, P("triangle").edges)
    assert judges.four_cycle_embeddings(g) == judges.brute_force(g, 4, P("4-cycle").edges)
    assert judges.clique_embeddings(g, 4) == judges.brute_force(g, 4, P("4-clique").edges)
    assert judges.star_embeddings(g, 3) == judges.brute_force(g, 4, P("3-star").edges)
    assert judges.wedge_embeddings(g) == judges.brute_force(g, 3, P("wedge").edges)
    for name in ["house", "5-cycle", "diamond", "4-path"]:
        p = P(name)
        assert judges.backtrack(g, p.k, p.edges) == judges.brute_force(g, p.k, p.edges)


def test_closed_forms_on_special_graphs():
    P = synth.named_pattern
    for n in [5, 6, 7]:
        kn = synth.complete_graph(n)
        for k in [3, 4, 5]:
            assert judges.clique_embeddings(kn, k) == math.perm(n, k)
            assert judges.backtrack(kn, k, synth.patterns.clique(k).edges) == math.perm(n, k)
    for n in [5, 6, 7, 8]:
        ring = synth.ring_graph(n)
        assert judges.backtrack(ring, n, synth.patterns.cycle(n).edges) == 2 * n  # one copy, |Aut| = 2n
        assert judges.backtrack(ring, 4, synth.patterns.path(4).edges) == 2 * n  # n copies of P4, |Aut| = 2
        assert judges.triangle_embeddings(ring) == 0
    kab = synth.complete_bipartite(4, 5)
    assert judges.four_cycle_embeddings(kab) == 8 * math.comb(4, 2) * math.comb(5, 2)
    st = synth.star_graph(6)
    assert judges.star_embeddings(st, 4) == math.perm(6, 4)
    assert judges.backtrack(st, 5, P("4-star").edges) == math.perm(6, 4)


# ------------------------------------------------------------ tables

def test_tables_degree_and_neighbour_degree_sum():
    g = synth.chung_lu(n=500, m=3000, seed=2)
    t = oracle.Tables(g, cv_seed=3)
    d = g.degrees()
    assert np.array_equal(t.deg, d)
    rows = np.repeat(np.arange(g.n), d)
    s2 = np.bincount(rows, weights=d[g.nbr.astype(np.int64)], minlength=g.n)
    assert np.array_equal(t.s2, s2.astype(np.uint64))


def test_exact_cv_is_local_triangle_count():
    g = synth.chung_lu(n=400, m=3000, seed=4)
    t = oracle.Tables(g, exact_cv=True)
    A = judges._adjacency(g)
    tri = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() / 2
    assert np.array_equal(t.hits, tri.astype(np.uint64))
    d = g.degrees()
    assert np.array_equal(t.trials, (d * (d - 1) // 2).astype(np.uint64))


def test_sampled_cv_is_unbiased():
    # Ordered pairs of distinct neighbours drawn uniformly: E[hits/d] = C_v.
    g = synth.chung_lu(n=300, m=2500, seed=5)
    ex = oracle.Tables(g, exact_cv=True).cv()
    acc = np.zeros(g.n)
    reps = 60
    for s in range(reps):
        acc += oracle.Tables(g, cv_seed=1000 + s).cv()
    d = g.degrees()
    sel = d >= 20
    mean = acc[sel] / reps
    # Standard error of a mean of reps * d Bernoulli(C_v) trials is <= 0.5/sqrt(reps*d).
    se = 0.5 / np.sqrt(reps * d[sel])
    assert np.all(np.abs(mean - ex[sel]) < 5 * se + 1e-9)


@pytest.mark.parametrize("exact_cv", [False, True])
def test_tables_at_matches_full_tables(exact_cv):
    g = synth.chung_lu(n=500, m=3000, seed=8)
    t = oracle.Tables(g, cv_seed=11, exact_cv=exact_cv)
    vs = np.array([0, 1, 7, 250, 499, 3, 3], dtype=np.uint64)
    a = oracle.tables_at(g, vs, cv_seed=11, exact_cv=exact_cv)
    for k in ("deg", "s2", "hits", "trials", "la", "lc"):
        assert np.array_equal(a[k], getattr(t, k)[vs.astype(np.int64)]), k


def test_lc_clamp_and_la():
    g = synth.star_graph(5)  # centre has C_v = 0, leaves have degree 1
    t = oracle.Tables(g, cv_seed=1)
    assert np.all(t.lc == oracle.LC_MIN_DEFAULT)
    # centre: average neighbour degree 1 -> log 0; leaves: 5 -> log2(5)
    assert t.la[0] == 0
    assert abs(t.la[1] / 65536 - math.log2(5)) < 1e-3


def test_worked_example_terms():
    fx = _worked_example()
    n = fx["graph_vertices"]
    us = [a for a, _ in fx["graph_edges"]]
    vs = [b for _, b in fx["graph_edges"]]
    g = synth.csr_from_edges(n, us, vs)
    t = oracle.Tables(g, exact_cv=True)
    a = 0
    cv = Fraction(int(t.hits[a]), int(t.trials[a]))
    assert cv == Fraction(5, 15)
    tf1, ti1, tf2 = oracle.literal_terms(int(t.deg[a]), fx["expect_b"], fx["expect_f1"], fx["expect_ie"],
                                         fx["expect_f2"], float(cv), int(t.s2[a]))
    assert tf1 == pytest.approx(float(fx["expect_T_F1"]), rel=1e-15)
    assert ti1 == pytest.approx(float(fx["expect_T_I1"]), rel=1e-15)
    assert tf2 == pytest.approx(float(fx["expect_T_F2"]), rel=1e-15)


# ------------------------------------------------------------ exact tree (Theorem 2)

TREE_CASES = [(gi, name) for gi in range(len(SMALL_GRAPHS))
              for name in ["triangle", "4-cycle", "4-clique", "house", "4-star", "5-cycle", "diamond",
                           "tailed-triangle"]]


@pytest.mark.parametrize("gi,name", TREE_CASES)
def test_unbiased_exact_enumeration(gi, name):
    g = SMALL_GRAPHS[gi]
    p = synth.named_pattern(name)
    exact = judges.brute_force(g, p.k, p.edges)
    adj = g.adjacency_sets()
    for mode in MODES:
        c = compile_pattern(p.k, p.edges, mode=mode)
        for exact_cv in (True, False):
            t = oracle.Tables(g, cv_seed=17, exact_cv=exact_cv)
            s = oracle.Sampler(g, t, c, seed=3)
            r = enumerate_tree(s)
            assert r["p_total"] == 1
            assert r["ex"] == exact
            # successful trajectories are exactly the embeddings
            succ = set()
            for tau in r["success"]:
                m = [None] * p.k
                for i, v in enumerate(tau):
                    m[c["order"][i]] = v
                assert all(m[b] in adj[m[a]] for a, b in p.edges)
                succ.add(tuple(m))
            assert len(succ) == len(r["success"]) == exact


@pytest.mark.parametrize("terms", ["f1", "f1_i1"])
@pytest.mark.parametrize("name", ["triangle", "4-clique", "house", "5-cycle", "diamond"])
def test_unbiased_exact_enumeration_term_ablation(name, terms):
    """Theorem 2 holds for any proposal that only zeroes certain zeros: the
    incremental versions of f_approx are still unbiased."""
    for gi in (0, 3):
        g = SMALL_GRAPHS[gi]
        p = synth.named_pattern(name)
        exact = judges.brute_force(g, p.k, p.edges)
        c = compile_pattern(p.k, p.edges, mode="always")
        s = oracle.Sampler(g, oracle.Tables(g, cv_seed=5), c, seed=3, terms=terms)
        r = enumerate_tree(s)
        assert r["p_total"] == 1 and r["ex"] == exact


@pytest.mark.parametrize("name", ["triangle", "4-clique", "house", "5-cycle", "diamond"])
def test_unbiased_exact_enumeration_learned_tables(name):
    """Theorem 2 with arbitrary learned tables: the pick and the importance
    factor use the same integer weights, so E[X] equals the exact count for
    any table; certain zeros (d(v) - |B| < |F1|) stay zero whatever the
    table says there; and the weights follow the table's order (a table
    ignored in favour of f_approx, or consulted for a certain zero, fails)."""
    rng = np.random.Generator(np.random.PCG64(11 + len(name)))
    for gi in (0, 3, 4):
        g = SMALL_GRAPHS[gi]
        p = synth.named_pattern(name)
        exact = judges.brute_force(g, p.k, p.edges)
        c = compile_pattern(p.k, p.edges, mode="learned")
        deg = np.diff(g.off).astype(np.int64)
        tabs = {}
        for i, st in enumerate(c["steps"]):
            if st["decision"] and st["f1"] > 0:
                t = rng.integers(-(8 << 16), 8 << 16, size=g.n).astype(np.int32)
                # the highest values of all at the vertices that cannot extend
                t[deg < st["b"] + st["f1"]] = 30 << 16
                tabs[i] = t
        assert tabs, name
        s = oracle.Sampler(g, oracle.Tables(g, cv_seed=5), c, seed=3, learned=tabs)
        r = enumerate_tree(s)
        assert r["p_total"] == 1 and r["ex"] == exact, (name, gi)
        prefixes = {tuple(tau[:i]) for tau in r["success"] for i in range(p.k)} | {()}
        for tau in prefixes:
            i = len(tau)
            if i not in tabs:
                continue
            st = c["steps"][i]
            vs, ws = s.step_distribution(i, list(tau))
            vs = vs.astype(np.int64)
            ws = ws.astype(np.int64)
            cz = deg[vs] < st["b"] + st["f1"]
            assert (ws[cz] == 0).all(), (name, gi, tau)
            live = ~cz & (ws > 0)
            lt = tabs[i][vs[live]].astype(np.int64)
            order = np.argsort(lt, kind="stable")
            assert (np.diff(ws[live][order]) >= 0).all(), (name, gi, tau)


def test_term_ablation_drops_the_right_factor():
    """Step 1 of the diamond has signature (b, f1, ie, f2) = (0, 3, 2, 0) and
    of the house (0, 3, 1, 2): T[F1] is d(d-1)(d-2) / 3! (its log is the sum
    of the three log2fx terms; the 3! cancels), T[I1] adds ie*LC and T[F2]
    adds f2*LA (Eq. probability_function).  The ablated versions keep
    exactly the leading factors."""
    g = synth.chung_lu(n=60, m=300, seed=4)
    t = oracle.Tables(g, cv_seed=2)
    d = np.diff(g.off).astype(np.int64)
    f1_part = np.array([sum(oracle.log2fx(int(x) - j) for j in range(3)) if x >= 3 else 0 for x in d])
    cz = d < 3
    for name, ie, f2 in (("diamond", 2, 0), ("house", 1, 2)):
        p = synth.named_pattern(name)
        c = compile_pattern(p.k, p.edges, mode="always")
        st = c["steps"][0]
        assert (st["b"], st["f1"], st["ie"], st["f2"]) == (0, 3, ie, f2)
        lw = {terms: oracle.Sampler(g, t, c, seed=0, terms=terms).log_weights(0) for terms in oracle.TERMS}
        for terms, expect in (("f1", f1_part), ("f1_i1", f1_part + ie * t.lc),
                              ("all", f1_part + ie * t.lc + f2 * t.la)):
            got = lw[terms]
            assert np.all(got[cz] == np.iinfo(np.int32).min)
            assert np.array_equal(got[~cz], expect[~cz].astype(np.int32)), terms


def test_kstar_first_step_is_ideal_zero_variance():
    # Sec. 3.2: drawing the centre with probability proportional to C(d, k)
    # makes every sample return k! * sum_v C(d(v), k) (zero variance).
    g = synth.chung_lu(n=40, m=110, seed=9)
    for leaves in (3, 4):
        p = synth.patterns.star(leaves)
        c = compile_pattern(p.k, p.edges, mode="switch")
        t = oracle.Tables(g, cv_seed=1)
        s = oracle.Sampler(g, t, c, seed=1)
        exact = judges.star_embeddings(g, leaves)
        cv = t.cv()
        r = enumerate_tree(s, literal_cv=cv)
        assert r["ex"] == exact
        assert r["ex2"] == r["ex"] ** 2  # literal weights: zero variance exactly
        _, xs, _ = s.run(0, 3000, want_x=True)
        nz = xs[xs != 0]
        assert nz.size == xs.size
        # integer weights: spread bounded by the Q16 encoding
        assert np.max(np.abs(nz / exact - 1)) < 5e-3


def _triangle_eta(g, v1, v2, cv):
    """Eq. alpha-def for a successful trajectory (v1, v2, v3)."""
    adj = g.adjacency_sets()
    d = g.degrees()
    s = sum(d[v] - 1 for v in adj[v1])
    common = len(adj[v1] & adj[v2])
    return (s * common / (d[v2] - 1)) / (d[v1] * (d[v1] - 1) * cv[v1]) - 1


def test_triangle_multiplicative_error_closed_forms():
    g = synth.chung_lu(n=40, m=180, seed=3)
    p = synth.named_pattern("triangle")
    C = judges.triangle_embeddings(g)
    assert C > 0
    t = oracle.Tables(g, exact_cv=True)
    cv = t.cv()
    adj = g.adjacency_sets()
    # f_approx with exact C_v: X = C (1 + eta_i) on every successful trajectory.
    c = compile_pattern(p.k, p.edges, mode="switch")
    s = oracle.Sampler(g, t, c, seed=2)
    recs = s.records(np.arange(4000))
    ok = recs[recs["fail_step"] < 0]
    assert ok.size > 100
    tree = enumerate_tree(s, literal_cv=cv)
    for tau in tree["success"][:200]:
        v1, v2, _ = tau
        p1 = Fraction(1)
        # X of the literal sampler is 1/p along the trajectory
        for i in range(3):
            vv, ww = s.step_distribution_literal(i, list(tau[:i]), cv)
            w = {int(a): Fraction(float(b)) for a, b in zip(vv, ww)}
            p1 *= w[tau[i]] / sum(w.values())
        x = float(1 / p1)
        assert x == pytest.approx(C * (1 + _triangle_eta(g, v1, v2, cv)), rel=1e-9)
    # the integer-encoded sampler stays within the encoding error of it
    for r in ok[:500]:
        v1, v2 = int(r["v"][0]), int(r["v"][1])
        assert r["x"] == pytest.approx(C * (1 + _triangle_eta(g, v1, v2, cv)), rel=2e-2)
    # f_uniform (NS-prune without symmetry breaking): X = 2|E| |N(v1) & N(v2)|.
    cu = compile_pattern(p.k, p.edges, mode="uniform")
    su = oracle.Sampler(g, t, cu, seed=2)
    recs = su.records(np.arange(3000))
    for r in recs[recs["fail_step"] < 0]:
        v1, v2 = int(r["v"][0]), int(r["v"][1])
        assert r["x"] == 2 * g.num_edges * len(adj[v1] & adj[v2])


# ------------------------------------------------------------ statistical unbiasedness

@pytest.mark.parametrize("name", ["triangle", "4-cycle", "4-clique"])
def test_unbiased_over_many_seeds(name):
    """Mean over 10^4 seeds (100 samples each) lies in the 99% CI of the
    exact count."""
    g = synth.chung_lu(n=300, m=2000, seed=11)
    p = synth.named_pattern(name)
    exact = judges.backtrack(g, p.k, p.edges)
    t = oracle.Tables(g, cv_seed=5)
    for mode in MODES:
        c = compile_pattern(p.k, p.edges, mode=mode)
        means = []
        s = oracle.Sampler(g, t, c, seed=0)
        for seed in range(10000):
            s.seed = seed
            st, _, _ = s.run(0, 100)
            means.append(st.mean)
        means = np.array(means)
        m = means.mean()
        se = means.std(ddof=1) / math.sqrt(means.size)
        assert abs(m - exact) <= 2.5758293035489004 * se, (mode, m, exact, se)


# ------------------------------------------------------------ sampler mechanics

def test_record_factors_match_step_distribution():
    g = synth.chung_lu(n=200, m=1200, seed=6)
    t = oracle.Tables(g, cv_seed=2)
    for name in ["house", "4-clique", "5-cycle"]:
        p = synth.named_pattern(name)
        for mode in MODES:
            c = compile_pattern(p.k, p.edges, mode=mode)
            s = oracle.Sampler(g, t, c, seed=9)
            recs = s.records(np.arange(300))
            for r in recs:
                steps = int(r["steps"])
                x = None
                for i in range(steps):
                    vv, ww = s.step_distribution(i, [int(a) for a in r["v"][:i]])
                    w = dict(zip(vv.tolist(), ww.tolist()))
                    assert int(r["num"][i]) == sum(w.values())
                    assert int(r["den"][i]) == w[int(r["v"][i])] > 0
                    f = float(int(r["num"][i])) / float(int(r["den"][i]))
                    x = f if x is None else x * f
                if r["fail_step"] >= 0:
                    assert r["x"] == 0.0
                    vv, ww = s.step_distribution(steps, [int(a) for a in r["v"][:steps]])
                    assert int(ww.sum()) == 0
                else:
                    assert steps == p.k and r["x"] == x


def test_no_embeddings_gives_zero():
    g = synth.ring_graph(12)
    p = synth.named_pattern("triangle")
    for mode in MODES:
        c = compile_pattern(p.k, p.edges, mode=mode)
        s = oracle.Sampler(g, oracle.Tables(g, cv_seed=1), c, seed=1)
        st, xs, _ = s.run(0, 500, want_x=True)
        assert st.mean == 0.0 and np.all(xs == 0) and eps_hat(st.n, st.mean, st.m2, 0.05) == math.inf


def test_empty_graph_gives_zero():
    g = synth.csr_from_edges(10, [], [])
    p = synth.named_pattern("triangle")
    for mode in MODES:
        c = compile_pattern(p.k, p.edges, mode=mode)
        s = oracle.Sampler(g, oracle.Tables(g), c, seed=1)
        st, xs, _ = s.run(0, 100, want_x=True)
        assert np.all(xs == 0)


def test_all_candidates_certain_zero():
    # 4-clique on a graph with max degree 2: the first weighted step has no
    # vertex with d >= 3, so every sample returns 0.
    g = synth.ring_graph(10)
    p = synth.named_pattern("4-clique")
    c = compile_pattern(p.k, p.edges, mode="switch")
    s = oracle.Sampler(g, oracle.Tables(g), c, seed=1)
    assert s.Q1 == 0
    _, xs, recs = s.run(0, 50, want_x=True, want_records=True)
    assert np.all(xs == 0) and np.all(recs["fail_step"] == 0)


def test_complete_graph_cliques_are_deterministic():
    # On K_n every k-clique trajectory succeeds; all weights tie, so every
    # sample returns n!/(n-k)! exactly.
    g = synth.complete_graph(7)
    for k in (3, 4, 5):
        p = synth.patterns.clique(k)
        for mode in MODES:
            c = compile_pattern(p.k, p.edges, mode=mode)
            s = oracle.Sampler(g, oracle.Tables(g, exact_cv=True), c, seed=1)
            _, xs, _ = s.run(0, 200, want_x=True)
            assert np.all(xs == math.perm(7, k))


def test_ring_cycles():
    # On the ring C_n the n-cycle has 2n embeddings and every trajectory
    # succeeds with probability 1 after the first pick in uniform mode.
    n = 8
    g = synth.ring_graph(n)
    p = synth.patterns.cycle(n)
    c = compile_pattern(p.k, p.edges, mode="uniform")
    s = oracle.Sampler(g, oracle.Tables(g), c, seed=4)
    _, xs, _ = s.run(0, 300, want_x=True)
    # step 1: 2|E|/d = n; step 2: two neighbours; later steps: one candidate
    assert np.all(xs == 2 * n)


# ------------------------------------------------------------ Algorithm 1

def test_z_values():
    assert z_value(0.05) == pytest.approx(1.959963984540054, abs=1e-12)
    assert z_value(0.01) == pytest.approx(2.5758293035489004, abs=1e-12)


def test_welford_matches_algorithm1_formulas():
    g = synth.chung_lu(n=300, m=2000, seed=11)
    p = synth.named_pattern("house")
    c = compile_pattern(p.k, p.edges)
    s = oracle.Sampler(g, oracle.Tables(g, cv_seed=5), c, seed=8)
    st, xs, _ = s.run(0, 5000, want_x=True)
    n, mu, var = direct_stats([float(x) for x in xs])
    assert st.n == n
    assert st.mean == pytest.approx(mu, rel=1e-12)
    assert st.m2 / st.n == pytest.approx(var, rel=1e-6)
    e = eps_hat(st.n, st.mean, st.m2, 0.05)
    assert e == pytest.approx(1.959963984540054 * math.sqrt(var) / (math.sqrt(n) * mu), rel=1e-6)


def test_run_to_eps_stop_depends_only_on_prefix():
    g = synth.chung_lu(n=300, m=2000, seed=11)
    p = synth.named_pattern("triangle")
    c = compile_pattern(p.k, p.edges)
    t = oracle.Tables(g, cv_seed=5)
    s = oracle.Sampler(g, t, c, seed=8)
    st, conv = run_to_eps(s, 0.05, 0.05, batch=256, min_samples=512, budget=1 << 20)
    assert conv and st.n % 256 == 0
    # the same stream checked in one go gives the same statistics
    st2, _, _ = oracle.Sampler(g, t, c, seed=8).run(0, st.n)
    assert st2.mean == st.mean and st2.m2 == st.m2
    # and the batch before it had not converged
    st3, _, _ = oracle.Sampler(g, t, c, seed=8).run(0, st.n - 256)
    assert st.n - 256 < 512 or eps_hat(st3.n, st3.mean, st3.m2, 0.05) > 0.05


# ------------------------------------------------------------ ideal first step and KL divergence

def _kl(ideal, q, total):
    """KL(f_ideal || f) with f(v) = q[v] / total; f must cover the ideal's support."""
    p = ideal.astype(np.float64) / ideal.sum()
    f = q.astype(np.float64) / float(total)
    m = p > 0
    assert np.all(f[m] > 0)
    return float(np.sum(p[m] * np.log(p[m] / f[m])))


def test_rooted_counts_closed_forms():
    g = synth.chung_lu(n=80, m=400, seed=6)
    d = np.diff(g.off).astype(np.int64)
    t = oracle.Tables(g, exact_cv=True)
    tri = synth.named_pattern("triangle")
    r = judges.rooted_counts(g, 3, tri.edges, [0, 1, 2])
    assert np.array_equal(r, 2 * t.hits.astype(np.int64))  # ordered pairs of adjacent neighbours
    star = synth.patterns.star(3)
    r = judges.rooted_counts(g, 4, star.edges, [0, 1, 2, 3])  # centre first
    assert np.array_equal(r, d * (d - 1) * (d - 2))
    for name in ("4-clique", "house", "4-path"):
        p = synth.named_pattern(name)
        c = compile_pattern(p.k, p.edges)
        r = judges.rooted_counts(g, p.k, p.edges, c["order"])
        assert int(r.sum()) == judges.backtrack(g, p.k, p.edges)


def test_first_step_kl_divergence_from_ideal():
    """The paper's analysis of the approximate distribution, on a skewed
    synthetic graph: the triangle's and the k-star's first steps are ideal
    up to the Q16 encoding (and the triangle's clamp of C_v); every f_approx is closer to f_ideal than the
    edge-uniform step; T[I1] is what makes the 4-clique close and T[F2] the
    4-path."""
    g = synth.chung_lu(n=300, m=1500, seed=4)
    d = np.diff(g.off).astype(np.int64)
    t = oracle.Tables(g, exact_cv=True)
    kl = {}
    for name in ("triangle", "3-star", "4-clique", "4-path", "diamond", "house"):
        p = synth.named_pattern(name)
        c = compile_pattern(p.k, p.edges, mode="always")
        ideal = judges.rooted_counts(g, p.k, p.edges, c["order"])
        kl[name] = {"uniform": _kl(ideal, d, int(d.sum()))}
        for terms in oracle.TERMS:
            s = oracle.Sampler(g, t, c, seed=0, terms=terms)
            kl[name][terms] = _kl(ideal, s.q1, s.Q1)
    print(kl)
    # triangle: the c_min clamp gives triangle-free vertices a small weight
    assert kl["triangle"]["all"] < 1e-4 and kl["3-star"]["all"] < 1e-6
    for name in kl:
        assert kl[name]["all"] < kl[name]["uniform"], name
    assert kl["4-clique"]["f1_i1"] < 0.5 * kl["4-clique"]["f1"]
    assert kl["4-path"]["all"] < 0.5 * kl["4-path"]["f1_i1"]


# ------------------------------------------------------------ degree orientation for cliques

def test_orientation_keeps_each_edge_once_in_degree_order():
    g = synth.chung_lu(n=300, m=1500, seed=3)
    o = oracle.orient(g)
    d = np.diff(g.off).astype(np.int64)
    assert o.n == g.n and o.nnz * 2 == g.nnz
    key = lambda v: (int(d[v]), int(v))
    seen = set()
    for v in range(o.n):
        row = o.nbr[int(o.off[v]):int(o.off[v + 1])]
        assert np.all(np.diff(row.astype(np.int64)) > 0)
        for w in row.tolist():
            assert key(v) < key(w)  # acyclic: every edge goes up the (degree, id) order
            seen.add((min(v, w), max(v, w)))
    und = {(v, int(w)) for v in range(g.n) for w in g.nbr[int(g.off[v]):int(g.off[v + 1])] if v < int(w)}
    assert seen == und


@pytest.mark.parametrize("k", [3, 4, 5])
def test_oriented_clique_sampler_is_unbiased_exactly(k):
    """Theorem 2 on the DAG: each k-clique is one trajectory, so E[X] is the
    clique count (exact rationals over the whole sampling tree)."""
    p = synth.patterns.clique(k)
    for gi in (0, 1, 3, 4):
        g = SMALL_GRAPHS[gi]
        cliques = judges.brute_force(g, k, p.edges) // math.factorial(k)
        o = oracle.orient(g)
        for mode in MODES:
            c = compile_pattern(p.k, p.edges, mode=mode)
            for exact_cv in (True, False):
                t = oracle.Tables(o, cv_seed=4, exact_cv=exact_cv, adjacency=g)
                r = enumerate_tree(oracle.Sampler(o, t, c, seed=1, oriented=True))
                assert r["p_total"] == 1 and r["ex"] == cliques, (gi, mode, exact_cv)


def test_oriented_tables_count_out_neighbours():
    g = synth.chung_lu(n=200, m=1200, seed=9)
    o = oracle.orient(g)
    t = oracle.Tables(o, exact_cv=True, adjacency=g)
    adj = g.adjacency_sets()
    dout = np.diff(o.off).astype(np.int64)
    assert np.array_equal(t.deg.astype(np.int64), dout)
    for v in range(0, g.n, 7):
        out = o.nbr[int(o.off[v]):int(o.off[v + 1])].tolist()
        pairs = sum(1 for a, b in itertools.combinations(out, 2) if b in adj[a])
        assert int(t.hits[v]) == pairs
        assert int(t.trials[v]) == len(out) * (len(out) - 1) // 2


def test_degrees_only_tables_serve_uniform_plans():
    """A uniform plan, and a star's weighted plans, read only the degrees:
    their records with the degrees-only tables (other entries null) equal
    those with the full tables, so every pin of these samplers carries over
    to them; the degrees are the row lengths."""
    g = synth.chung_lu(n=2000, m=12_000, gamma=2.1, seed=4)
    full = oracle.Tables(g, cv_seed=3)
    deg = oracle.Tables.degrees_only(g)
    assert np.array_equal(deg.deg, np.diff(g.off).astype(np.uint32))
    assert np.array_equal(deg.deg, full.deg)
    assert deg.la is None and deg.lc is None and deg.s2 is None
    idx = np.concatenate([np.arange(2000), [2 ** 33 + 3, 2 ** 63 + 11]]).astype(np.uint64)
    for name in ("5-clique", "6-cycle", "house", "4-star", "chordal-7-cycle"):
        p = synth.named_pattern(name)
        c = compile_pattern(p.k, p.edges, mode="uniform")
        a = oracle.Sampler(g, full, c, seed=5).records(idx)
        b = oracle.Sampler(g, deg, c, seed=5).records(idx)
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), name
        assert (a["fail_step"] < 0).any(), name
    # a star's weighted plans read the degrees alone: the centre first,
    # weighted by T[F1] only (no I1, no F2), the leaves trivial
    for name in ("4-star", "3-star"):
        p = synth.named_pattern(name)
        for mode in ("switch", "always"):
            c = compile_pattern(p.k, p.edges, mode=mode)
            weighted = [s for s in c["steps"] if s["decision"] == 1 and s["f1"] > 0]
            assert weighted and all(s["ie"] == 0 and s["f2"] == 0 for s in weighted), (name, mode)
            assert c["steps"][0] in weighted
            a = oracle.Sampler(g, full, c, seed=5)
            b = oracle.Sampler(g, deg, c, seed=5)
            assert a.Q1 == b.Q1 > 0 and np.array_equal(a.q1, b.q1)
            ra, rb = a.records(idx), b.records(idx)
            assert np.array_equal(ra.view(np.uint8), rb.view(np.uint8)), (name, mode)
