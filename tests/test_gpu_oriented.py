"""GPU: degree orientation for clique patterns -- the oriented CSR, its
tables, the sampled records and estimates against the oracle and exact
clique counts."""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import judges
from oracle.pattern import compile_pattern

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2601_01388_amd")

MODES = ["uniform", "switch", "always"]


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
def c1(sess):
    g = synth.chung_lu(n=10000, m=100000, seed=1)
    G = sess.graph(g.off, g.nbr)
    say("orienting Chung-Lu 10k/100k")
    O = sess.orient(G)
    T = sess.tables(O, cv_seed=1)
    o = oracle.orient(g)
    OT = oracle.Tables(o, cv_seed=1, adjacency=g)
    yield g, G, O, T, o, OT
    T.close()
    O.close()
    G.close()


def test_oriented_csr_and_tables_parity(sess, c1):
    g, G, O, T, o, OT = c1
    off, nbr = O.csr()
    assert np.array_equal(off, o.off) and np.array_equal(nbr, o.nbr)
    got = T.export()
    for k in ("deg", "s2", "hits", "trials", "la", "lc"):
        assert np.array_equal(got[k], getattr(OT, k)), k


def test_oriented_csr_rmat16(sess):
    g = synth.rmat(16, 16, seed=16)
    G = sess.graph(g.off, g.nbr)
    O = sess.orient(G)
    off, nbr = O.csr()
    o = oracle.orient(g)
    assert np.array_equal(off, o.off) and np.array_equal(nbr, o.nbr)
    O.close()
    G.close()


@pytest.mark.parametrize("rowtab", ["off", "on"])
@pytest.mark.parametrize("k", [3, 4, 5])
def test_oriented_records_parity(sess, c1, k, rowtab):
    g, G, O, T, o, OT = c1
    p = synth.patterns.clique(k)
    idx = np.concatenate([np.arange(3000), np.array([2 ** 33 + 1, 2 ** 62 + 9])]).astype(np.uint64)
    for mode in MODES:
        say(f"oriented records {k}-clique {mode} rowtab={rowtab}")
        got = sess.dump(O, T, p, 7, idx, mode=mode, rowtab=rowtab, pattern_id=1)
        ref = oracle.Sampler(o, OT, compile_pattern(p.k, p.edges, mode=mode), seed=7, pattern_id=1,
                             oriented=True).records(idx)
        for f in ("v", "num", "den", "steps", "fail_step"):
            assert np.array_equal(got[f], ref[f]), (mode, f)
        assert np.array_equal(got["x"], ref["x"]), mode


@pytest.mark.parametrize("k", [3, 4, 5])
def test_oriented_estimates_against_exact_cliques(sess, c1, k):
    g, G, O, T, o, OT = c1
    p = synth.patterns.clique(k)
    cliques = judges.clique_embeddings(g, k) // math.factorial(k)
    for mode in ("switch", "uniform"):
        r = sess.estimate(O, T, p, 1 << 21, 3, mode=mode)
        se = math.sqrt(r.variance / r.n) / math.factorial(k)
        assert abs(r.copies - cliques) <= 5 * se + 1e-9 * cliques, (mode, r.copies, cliques, se)
        assert r.estimate == pytest.approx(r.copies * math.factorial(k), rel=1e-12)


def test_oriented_rejects_non_cliques(sess, c1):
    g, G, O, T, o, OT = c1
    with pytest.raises(A.AgisError) as e:
        sess.estimate(O, T, synth.named_pattern("house"), 1000, 1)
    assert e.value.code == A.AGIS_E_UNSUPPORTED


def test_oriented_rmat20_full_size_sampled_parity(sess):
    """The bench's clique workload at full size: R-MAT scale 20 oriented on
    the GPU, its CSR and tables compared whole with the oracle's, records of
    the 4- and 5-clique compared on indices sampled from [0, 10^8), and the
    oriented 5-clique estimate against the symmetric graph's."""
    g = synth.rmat(20, 16, seed=20)
    say(f"R-MAT-20 orient n={g.n} nnz={g.nnz}")
    G = sess.graph(g.off, g.nbr)
    O = sess.orient(G)
    T = sess.tables(O, cv_seed=1)
    o = oracle.orient(g)
    off, nbr = O.csr()
    assert np.array_equal(off, o.off) and np.array_equal(nbr, o.nbr)
    say("R-MAT-20 oriented tables compare")
    OT = oracle.Tables(o, cv_seed=1, adjacency=g)
    got = T.export()
    for k in ("deg", "s2", "hits", "trials", "la", "lc"):
        assert np.array_equal(got[k], getattr(OT, k)), k
    rng = np.random.Generator(np.random.PCG64(21))
    idx = np.sort(rng.integers(0, 10 ** 8, size=400, dtype=np.uint64))
    for k in (4, 5):
        p = synth.patterns.clique(k)
        ref = oracle.Sampler(o, OT, compile_pattern(p.k, p.edges, mode="switch"), seed=7,
                             oriented=True).records(idx)
        for rowtab in ("off", "on"):
            say(f"R-MAT-20 oriented records {k}-clique rowtab={rowtab}")
            rec = sess.dump(O, T, p, 7, idx, mode="switch", rowtab=rowtab)
            for f in ("v", "num", "den", "steps", "fail_step"):
                assert np.array_equal(rec[f], ref[f]), (k, rowtab, f)
            assert np.array_equal(rec["x"], ref["x"]), (k, rowtab)
    say("R-MAT-20 5-clique: oriented vs symmetric estimate")
    p = synth.patterns.clique(5)
    TS = sess.tables(G, cv_seed=1)
    ro = sess.estimate(O, T, p, 1 << 22, 7, mode="switch")
    rs = sess.estimate(G, TS, p, 1 << 22, 8, mode="switch")
    se = math.sqrt(ro.variance / ro.n + rs.variance / rs.n)  # both in embeddings
    assert abs(ro.estimate - rs.estimate) <= 5 * se, (ro.estimate, rs.estimate, se)
    TS.close()
    T.close()
    O.close()
    G.close()


@pytest.mark.parametrize("k", [3, 4, 5])
def test_oriented_production_estimates_match_oracle(sess, c1, k):
    """The production kernel on the DAG (count-only last step, pair-hub
    table of out-neighbourhoods) against the oracle's mean over the same
    sample indices: the estimate is k! times it."""
    g, G, O, T, o, OT = c1
    p = synth.patterns.clique(k)
    n = 50_000
    for mode in ("switch", "uniform"):
        r = sess.estimate(O, T, p, n, 7, mode=mode)
        st, _, _ = oracle.Sampler(o, OT, compile_pattern(p.k, p.edges, mode=mode), seed=7, oriented=True).run(0, n)
        assert r.n == n
        exact = math.factorial(k) * st.mean
        assert abs(r.estimate - exact) <= 1e-9 * abs(exact), (mode, r.estimate, exact)
