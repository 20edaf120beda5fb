"""GPU: concentrations of all connected k-vertex patterns from one batched
estimate per pattern, against exact counts (the oracle's backtracking
counter) on a small skewed graph."""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import concentration as conc
from oracle import judges
from oracle.pattern import automorphisms

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2601_01388_amd")


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


@pytest.mark.parametrize("k,n,m", [(4, 400, 2400), (5, 250, 1200)])
def test_concentrations_against_exact_counts(sess, k, n, m):
    g = synth.chung_lu(n=n, m=m, seed=5)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    say(f"batched estimates, k={k}")
    out = sess.concentrations(G, T, k, 1 << 21, 9, mode="switch")
    tup = out["patterns"]
    assert len(tup) == len(synth.patterns.connected_patterns(k))
    say(f"exact copies of {len(tup)} patterns on k={k}")
    exact = [judges.backtrack(g, kk, e) // automorphisms(kk, e) for kk, e in tup]
    for (kk, e), r, x in zip(tup, out["results"], exact):
        se = math.sqrt(r.variance / r.n) / r.aut
        assert abs(r.copies - x) <= 5 * se + 1e-9 * max(x, 1), (e, r.copies, x, se)
    exact_ce = conc.normalise(exact)
    assert conc.variation_distance(out["conc_edge"], exact_ce) < 0.01
    exact_ci = conc.normalise(conc.induced_from_copies(tup, exact))
    assert conc.variation_distance(out["conc_induced"], exact_ci) < 0.02
    T.close()
    G.close()
