"""GPU parity: the HIP library against the CPU oracle, through the C-ABI.

Bar: integer work (tables, vertex choices, integer factors, failure step)
bit-exact; per-sample FP64 weights equal (relative 1e-12 is the stated
tolerance, the implementation reproduces the IEEE result exactly);
estimates within relative 1e-9 (only the FP64 reduction order differs).
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import judges
from oracle.estimator import run_to_eps
from oracle.pattern import compile_pattern

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2601_01388_amd")

MODES = ["uniform", "switch", "always"]
SEED = 7
CV_SEED = 1


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sess():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_01388_amd.session import Session
    s = Session(0)
    yield s
    s.close()


@pytest.fixture(scope="module")
def c1():
    return synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)


def _compare_tables(got, ref):
    for f in ("deg", "s2", "hits", "trials", "la", "lc"):
        a = got[f]
        b = getattr(ref, f)
        assert a.shape == b.shape
        bad = np.flatnonzero(a.astype(np.int64) != b.astype(np.int64))
        assert bad.size == 0, (f, bad[:10], a[bad[:10]], b[bad[:10]])


GRAPHS = {
    "tiny8": lambda: synth.graphs.tiny_graph(8, 0.5, 0),
    "skew9": lambda: synth.graphs.skewed_tiny_graph(9, seed=1),
    "K7": lambda: synth.complete_graph(7),
    "star6": lambda: synth.star_graph(6),
    "cl500": lambda: synth.chung_lu(n=500, m=4000, seed=3),
}


@pytest.mark.parametrize("gname", list(GRAPHS))
@pytest.mark.parametrize("exact", [False, True])
def test_tables_parity_small(sess, gname, exact):
    g = GRAPHS[gname]()
    say(f"tables {gname} exact={exact}")
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=CV_SEED, exact_cv=exact)
    _compare_tables(T.export(), oracle.Tables(g, cv_seed=CV_SEED, exact_cv=exact))
    T.close()
    G.close()


@pytest.mark.parametrize("exact", [False, True])
def test_tables_parity_c1(sess, c1, exact):
    say(f"tables chung-lu 10k/100k exact={exact}")
    G = sess.graph(c1.off, c1.nbr)
    T = sess.tables(G, cv_seed=CV_SEED, exact_cv=exact)
    _compare_tables(T.export(), oracle.Tables(c1, cv_seed=CV_SEED, exact_cv=exact))


def _compare_records(got, ref, label):
    assert got.shape == ref.shape
    for f in ("steps", "fail_step"):
        bad = np.flatnonzero(got[f] != ref[f])
        assert bad.size == 0, (label, f, bad[:5], got[f][bad[:5]], ref[f][bad[:5]])
    for f in ("v", "num", "den"):
        bad = np.flatnonzero((got[f] != ref[f]).any(axis=1))
        assert bad.size == 0, (label, f, bad[:5], got[f][bad[:5]], ref[f][bad[:5]])
    # per-sample FP64 weights: same IEEE double (stated tolerance 1e-12 relative)
    x, y = got["x"], ref["x"]
    rel = np.abs(x - y) / np.maximum(np.abs(y), 1e-300)
    assert np.all((x == y) | (rel <= 1e-12)), (label, np.max(rel))
    assert np.array_equal(x, y), (label, "weights differ in the last bit", np.max(rel))


def _indices(m, rng_seed=0):
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    base = np.arange(m, dtype=np.uint64)
    far = rng.integers(0, 1 << 62, size=m // 4, dtype=np.uint64)
    edge = np.array([(1 << 32) - 1, 1 << 32, (1 << 63) - 1, (1 << 64) - 1], dtype=np.uint64)
    return np.concatenate([base, far, edge])


C1_PATTERNS = ["triangle", "4-cycle", "4-clique", "house", "5-cycle", "4-star", "diamond", "edge"]


@pytest.fixture(scope="module")
def c1_state(sess, c1):
    G = sess.graph(c1.off, c1.nbr)
    T = sess.tables(G, cv_seed=CV_SEED)
    OT = oracle.Tables(c1, cv_seed=CV_SEED)
    return G, T, OT


@pytest.mark.parametrize("rowtab", ["off", "on"])
@pytest.mark.parametrize("name", C1_PATTERNS)
@pytest.mark.parametrize("mode", MODES)
def test_records_parity_c1(sess, c1, c1_state, name, mode, rowtab):
    G, T, OT = c1_state
    p = synth.named_pattern(name)
    idx = _indices(3000, rng_seed=sum(name.encode()))
    say(f"records chung-lu {name} {mode} rowtab={rowtab} m={idx.size}")
    got = sess.dump(G, T, p, SEED, idx, mode=mode, pattern_id=5, rowtab=rowtab)
    c = compile_pattern(p.k, p.edges, mode=mode)
    ref = oracle.Sampler(c1, OT, c, seed=SEED, pattern_id=5).records(idx)
    _compare_records(got, ref, f"{name}/{mode}")


@pytest.mark.parametrize("rowtab", ["off", "on"])
@pytest.mark.parametrize("mode", ["uniform", "switch"])
@pytest.mark.parametrize("k", [6, 7, 8])
def test_records_parity_c1_long_paths(sess, c1, c1_state, k, mode, rowtab):
    """Paths of 6 to 8 vertices: single-backward steps with five to seven
    matched vertices, located in the row by the eight-lane search groups
    (the bench patterns use the sixteen-lane ones)."""
    G, T, OT = c1_state
    p = synth.patterns.path(k)
    idx = _indices(2000, rng_seed=100 + k)
    say(f"records chung-lu path({k}) {mode} rowtab={rowtab} m={idx.size}")
    got = sess.dump(G, T, p, SEED, idx, mode=mode, pattern_id=6, rowtab=rowtab)
    c = compile_pattern(p.k, p.edges, mode=mode)
    ref = oracle.Sampler(c1, OT, c, seed=SEED, pattern_id=6).records(idx)
    _compare_records(got, ref, f"path({k})/{mode}")


@pytest.mark.parametrize("rowtab", ["off", "on"])
@pytest.mark.parametrize("terms", ["f1", "f1_i1"])
@pytest.mark.parametrize("name", ["house", "4-clique", "5-cycle", "diamond"])
def test_records_parity_term_ablation(sess, c1, c1_state, name, terms, rowtab):
    G, T, OT = c1_state
    p = synth.named_pattern(name)
    idx = _indices(2000, rng_seed=7 + sum(name.encode()))
    say(f"records chung-lu {name} terms={terms} rowtab={rowtab} m={idx.size}")
    got = sess.dump(G, T, p, SEED, idx, mode="always", pattern_id=2, rowtab=rowtab, terms=terms)
    c = compile_pattern(p.k, p.edges, mode="always")
    ref = oracle.Sampler(c1, OT, c, seed=SEED, pattern_id=2, terms=terms).records(idx)
    _compare_records(got, ref, f"{name}/{terms}")


@pytest.mark.parametrize("name", ["triangle", "4-clique", "house", "4-cycle", "5-cycle"])
def test_step1_weights_parity(sess, c1, c1_state, name):
    """The first-step proposal the library exports equals the oracle's."""
    G, T, OT = c1_state
    p = synth.named_pattern(name)
    d = np.diff(c1.off).astype(np.int64)
    for mode in MODES:
        for terms in ("all", "f1", "f1_i1"):
            q1, total = sess.step1_weights(G, T, p, mode=mode, terms=terms)
            s = oracle.Sampler(c1, OT, compile_pattern(p.k, p.edges, mode=mode), seed=0, terms=terms)
            if s.Q1:
                assert total == s.Q1 and np.array_equal(q1, s.q1.astype(np.int64)), (mode, terms)
            else:  # edge-uniform first step
                assert total == c1.nnz and np.array_equal(q1, d), (mode, terms)


def test_records_shape_invariance(sess, c1, c1_state):
    """The same sample index gives the same record whatever the launch."""
    G, T, OT = c1_state
    p = synth.named_pattern("house")
    idx = np.arange(5000, dtype=np.uint64)
    say("records shape invariance")
    a = sess.dump(G, T, p, SEED, idx)
    for m in (1, 63, 65, 777):
        b = sess.dump(G, T, p, SEED, idx[:m])
        assert np.array_equal(a[:m].view(np.uint8), b.view(np.uint8))
    c = sess.dump(G, T, p, SEED, idx[::-1].copy())
    assert np.array_equal(np.ascontiguousarray(a[::-1]).view(np.uint8), c.view(np.uint8))


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "4-clique", "house"])
@pytest.mark.parametrize("mode", MODES)
def test_estimate_parity_c1(sess, c1, c1_state, name, mode):
    G, T, OT = c1_state
    p = synth.named_pattern(name)
    n = 200_000
    say(f"estimate chung-lu {name} {mode} n={n}")
    r = sess.estimate(G, T, p, n, SEED, mode=mode)
    r2 = sess.estimate(G, T, p, n, SEED, mode=mode, rowtab="off", check_every=12345, eps=1e-30)
    assert r2.n == n and r2.estimate == pytest.approx(r.estimate, rel=1e-12)
    c = compile_pattern(p.k, p.edges, mode=mode)
    st, _, _ = oracle.Sampler(c1, OT, c, seed=SEED).run(0, n)
    assert r.n == st.n and r.n_nonzero == st.nonzero
    assert r.estimate == pytest.approx(st.mean, rel=1e-9)
    assert r.variance == pytest.approx(st.m2 / st.n, rel=1e-9)
    assert r.aut == c["aut"] and r.copies == pytest.approx(st.mean / c["aut"], rel=1e-9)


def test_estimate_against_exact_counts_c1(sess, c1, c1_state):
    """10^6 samples per pattern and mode land within 99.9% CI of the exact count."""
    G, T, _ = c1_state
    exact = {"triangle": judges.triangle_embeddings(c1), "4-cycle": judges.four_cycle_embeddings(c1),
             "4-clique": judges.clique_embeddings(c1, 4)}
    for name, C in exact.items():
        for mode in MODES:
            say(f"exact-count check {name} {mode}")
            r = sess.estimate(G, T, synth.named_pattern(name), 1_000_000, SEED, mode=mode)
            se = math.sqrt(r.variance / r.n)
            assert abs(r.estimate - C) <= 3.29 * se + 1e-9 * C, (name, mode, r.estimate, C, se)


def test_run_to_eps_parity(sess, c1, c1_state):
    G, T, OT = c1_state
    p = synth.named_pattern("4-clique")
    for mode in MODES:
        say(f"run-to-eps chung-lu 4-clique {mode}")
        r = sess.estimate(G, T, p, 1 << 22, SEED, mode=mode, eps=0.02, delta=0.05, check_every=4096,
                          min_samples=8192)
        c = compile_pattern(p.k, p.edges, mode=mode)
        st, conv = run_to_eps(oracle.Sampler(c1, OT, c, seed=SEED), 0.02, 0.05, 4096, 8192, 1 << 22)
        assert bool(r.converged) == conv and r.n == st.n, (mode, r.n, st.n)
        assert r.estimate == pytest.approx(st.mean, rel=1e-9)


def test_edge_cases(sess):
    # graph without edges: every sample fails at step 0
    g = synth.csr_from_edges(5, [], [])
    say("edge case: empty graph")
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G)
    for mode in MODES:
        r = sess.estimate(G, T, synth.named_pattern("triangle"), 1000, 1, mode=mode)
        assert r.estimate == 0.0 and r.n == 1000 and r.n_nonzero == 0 and math.isinf(r.eps_hat)
    # no embeddings (ring has no triangle) and all-certain-zero first step
    ring = synth.ring_graph(50)
    say("edge case: ring")
    G2 = sess.graph(ring.off, ring.nbr)
    T2 = sess.tables(G2)
    OT2 = oracle.Tables(ring)
    for name in ("triangle", "4-clique", "5-cycle"):
        for mode in MODES:
            p = synth.named_pattern(name)
            got = sess.dump(G2, T2, p, 3, np.arange(300, dtype=np.uint64), mode=mode)
            ref = oracle.Sampler(ring, OT2, compile_pattern(p.k, p.edges, mode=mode), seed=3).records(np.arange(300))
            _compare_records(got, ref, f"ring/{name}/{mode}")
    # complete graph: every clique sample returns n!/(n-k)!
    k7 = synth.complete_graph(7)
    G3 = sess.graph(k7.off, k7.nbr)
    T3 = sess.tables(G3, exact_cv=True)
    for k in (3, 4, 5):
        r = sess.estimate(G3, T3, synth.patterns.clique(k), 999, 2, mode="always")
        assert r.estimate == math.perm(7, k) and r.variance == 0.0
    # ragged sample counts
    for n in (1, 63, 65, 4097):
        r = sess.estimate(G3, T3, synth.named_pattern("triangle"), n, 2)
        assert r.n == n


@pytest.mark.parametrize("case", ["unsorted", "duplicate", "self_loop", "asymmetric", "out_of_range", "bad_end"])
def test_invalid_csr_rejected(sess, case):
    g = synth.graphs.tiny_graph(8, 0.6, 1)
    off = g.off.copy()
    nbr = g.nbr.copy()
    r0 = slice(int(off[0]), int(off[1]))
    if case == "unsorted":
        row = nbr[r0].copy()
        nbr[r0] = row[::-1]
    elif case == "duplicate":
        nbr[int(off[0]) + 1] = nbr[int(off[0])]
    elif case == "self_loop":
        nbr[int(off[0])] = 0
    elif case == "asymmetric":
        nbr[int(off[1]) - 1] = 7 if nbr[int(off[1]) - 1] != 7 else 6
        nbr[r0] = np.sort(nbr[r0])
    elif case == "out_of_range":
        nbr[-1] = 100
    elif case == "bad_end":
        off[-1] = off[-1] - 2
    say(f"invalid CSR {case}")
    with pytest.raises(A.AgisError) as e:
        sess.graph(off, nbr)
    assert e.value.code == A.AGIS_E_INVALID_CSR


# --------------------------------------------------------------- R-MAT scale 20

@pytest.fixture(scope="module")
def rmat20():
    say("generating R-MAT scale 20")
    return synth.rmat(20, 16, seed=20)


C2_PATTERNS = ["5-clique", "5-cycle", "house", "4-star"]


def test_rmat20_full_size_sampled_parity(sess, rmat20):
    """Full-size graph, bench launch shape: tables compared whole, records
    compared on sampled indices spread over [0, 10^8)."""
    g = rmat20
    say(f"R-MAT-20 load n={g.n} nnz={g.nnz}")
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=CV_SEED)
    OT = oracle.Tables(g, cv_seed=CV_SEED)
    say("R-MAT-20 tables compare")
    _compare_tables(T.export(), OT)
    rng = np.random.Generator(np.random.PCG64(20))
    idx = np.sort(rng.integers(0, 10 ** 8, size=400, dtype=np.uint64))
    for name in C2_PATTERNS:
        p = synth.named_pattern(name)
        for mode in ("switch", "uniform"):
            ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode=mode), seed=SEED).records(idx)
            for rowtab in ("off", "on"):
                say(f"R-MAT-20 records {name} {mode} rowtab={rowtab}")
                got = sess.dump(G, T, p, SEED, idx, mode=mode, rowtab=rowtab)
                _compare_records(got, ref, f"rmat20/{name}/{mode}/{rowtab}")
    # 4-star has a closed form: k! * sum C(d, 4)
    say("R-MAT-20 4-star closed form")
    r = sess.estimate(G, T, synth.named_pattern("4-star"), 100_000, SEED, mode="switch")
    exact = judges.star_embeddings(g, 4)
    assert abs(r.estimate / exact - 1) < 0.01


def test_rmat20_estimates_match_oracle(sess, rmat20):
    """The production sampler as the bench runs it (count-only last steps,
    the pair-hub count table for common neighbours of two top hubs, row
    pick tables on and off, the lane sampler for the 4-star, the core-pair
    lists and pick tables of the cliques) against the
    oracle's mean over the same sample indices of the full-size graph (the
    oracle on all host threads, one sampler per thread)."""
    g = rmat20
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=CV_SEED)
    OT = oracle.Tables(g, cv_seed=CV_SEED, threads=0)
    for name, n in (("5-clique", 1 << 15), ("5-cycle", 1 << 17), ("house", 1 << 17), ("4-star", 1 << 16),
                    ("4-cycle", 1 << 17), ("triangle", 1 << 17), ("4-clique", 1 << 16), ("6-clique", 1 << 13),
                    ("chordal-7-cycle", 1 << 14)):
        p = synth.named_pattern(name)
        st, _ = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode="switch"), seed=SEED).run_parallel(0, n)
        for rowtab in ("on", "off"):
            say(f"R-MAT-20 estimate {name} n={n} rowtab={rowtab}")
            r = sess.estimate(G, T, p, n, SEED, mode="switch", rowtab=rowtab)
            assert r.n == n
            assert abs(r.estimate - st.mean) <= 1e-9 * abs(st.mean), (name, rowtab, r.estimate, st.mean)
    T.close()
    G.close()


# patterns of the seeded 32-pattern set whose weighted steps have two
# backward vertices: drawn through the core-pair pick tables, at step 2, 3
# or 4, over the pairs {0, 1}, {1, 2} and {0, 2}, with earlier matched
# vertices that may lie in the pair's list (12 has two such steps)
CORE_PICK_BATCH = [12, 14, 19, 22, 25, 28]


def test_rmat20_core_pick_steps_match_oracle(sess, rmat20):
    """Records on sampled indices and estimates (to rel 1e-9) of those
    patterns on the full-size graph, with row and pick tables on and off."""
    g = rmat20
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=CV_SEED)
    OT = oracle.Tables(g, cv_seed=CV_SEED, threads=0)
    pset = synth.random_pattern_set(32, seed=3)
    rng = np.random.Generator(np.random.PCG64(21))
    idx = np.sort(rng.integers(0, 10 ** 8, size=600, dtype=np.uint64))
    for which in CORE_PICK_BATCH:
        p = pset[which][0]
        c = compile_pattern(p.k, p.edges, mode="switch")
        S = oracle.Sampler(g, OT, c, seed=SEED, pattern_id=which)
        ref = S.records(idx, threads=0)
        st, _ = S.run_parallel(0, 1 << 14)
        for rowtab in ("on", "off"):
            say(f"R-MAT-20 batch pattern {which} (k={p.k}, {len(p.edges)} edges) rowtab={rowtab}")
            got = sess.dump(G, T, p, SEED, idx, mode="switch", pattern_id=which, rowtab=rowtab)
            _compare_records(got, ref, f"rmat20/batch{which}/{rowtab}")
            r = sess.estimate(G, T, p, 1 << 14, SEED, mode="switch", pattern_id=which, rowtab=rowtab)
            assert abs(r.estimate - st.mean) <= 1e-9 * abs(st.mean), (which, rowtab, r.estimate, st.mean)
    T.close()
    G.close()


@pytest.mark.parametrize("n", [70, 130])
def test_complete_graph_closed_forms_with_pair_hubs(sess, n):
    """On K_n (n >= 65) every vertex has a neighbourhood bitmap and is a pair
    hub, and every matched vertex lies in both lists of a two-list step, so
    the pair-hub count and rank selection must subtract each of them.  Every
    injective map is an embedding: each sample's X is n!/(n-k)! exactly,
    in every mode, and the records equal the oracle's."""
    g = synth.complete_graph(n)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=CV_SEED)
    OT = oracle.Tables(g, cv_seed=CV_SEED)
    idx = np.arange(2000, dtype=np.uint64)
    for name in ("triangle", "4-cycle", "house", "5-cycle", "diamond"):
        p = synth.named_pattern(name)
        exact = float(math.perm(n, p.k))
        for mode in ("switch", "uniform", "always"):
            say(f"K_{n} {name} {mode}")
            r = sess.estimate(G, T, p, 50_000, SEED, mode=mode)
            assert r.estimate == pytest.approx(exact, rel=1e-12), (name, mode, r.estimate, exact)
            got = sess.dump(G, T, p, SEED, idx, mode=mode)
            ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode=mode), seed=SEED).records(idx)
            _compare_records(got, ref, f"K{n}/{name}/{mode}")
    T.close()
    G.close()
