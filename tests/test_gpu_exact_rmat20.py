"""GPU estimates on the R-MAT scale 20 bench graph against its exact clique
counts (tests/golden/rmat20_clique_counts.txt, written by the oracle's
clique lister) and the 4-star closed form: the estimator is unbiased
(Theorem 2), so a long run lands within a few standard errors of the exact
count, on the symmetric graph and on its degree orientation."""

import math
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2601_01388_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat20_clique_counts.txt")


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def golden():
    out = {}
    if os.path.exists(GOLDEN):
        for line in open(GOLDEN):
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[int(k)] = int(v)
    return out


@pytest.fixture(scope="module")
def r20():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_01388_amd.session import Session
    say("R-MAT scale 20 (seed 20)")
    g = synth.rmat(20, 16, seed=20)
    s = Session(0)
    G = s.graph(g.off, g.nbr)
    T = s.tables(G, cv_seed=1)
    O = s.orient(G)
    TO = s.tables(O, cv_seed=1)
    yield g, s, G, T, O, TO
    TO.close()
    O.close()
    T.close()
    G.close()
    s.close()


def _check(r, exact, what):
    se = math.sqrt(r.variance / r.n)
    z = (r.estimate - exact) / se if se > 0 else 0.0
    say(f"{what}: estimate {r.estimate:.6g}, exact {exact}, z = {z:.2f}")
    assert abs(r.estimate - exact) <= 5 * se + 1e-12 * exact, (what, r.estimate, exact, se)


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("graph", ["symmetric", "oriented"])
def test_clique_estimates_match_exact_counts(r20, k, graph):
    g, s, G, T, O, TO = r20
    gold = golden()
    if k not in gold:
        pytest.skip(f"no exact {k}-clique count in {GOLDEN} yet")
    gg, tt = (G, T) if graph == "symmetric" else (O, TO)
    r = s.estimate(gg, tt, synth.patterns.clique(k), 1 << 24, 101 + k, mode="switch", pattern_id=k)
    _check(r, gold[k], f"{k}-clique on the {graph} graph")


def test_four_star_matches_closed_form(r20):
    g, s, G, T, O, TO = r20
    d = np.diff(g.off).astype(np.int64)
    exact = int(sum(math.perm(int(x), 4) for x in d[d >= 4]))
    r = s.estimate(G, T, synth.named_pattern("4-star"), 1 << 22, 5, mode="switch")
    _check(r, exact, "4-star")


def test_batch_to_eps_in_one_launch_equals_host_rounds(r20):
    """The bench's 32-pattern batch on this graph (seed 3, budgets
    log-uniform in [10^6, 10^9], +-1% at 95%, checks every 2^16 from 2^14):
    the one-launch run stops every pattern at the same sample count as the
    round-by-round run with the checks on the host, with the same estimate."""
    g, s, G, T, O, TO = r20
    pset = synth.random_pattern_set(32, seed=3)
    pats, budgets = [p for p, _ in pset], [b for _, b in pset]
    kw = dict(mode="switch", eps=0.01, delta=0.05, check_every=1 << 16, min_samples=1 << 14)
    dev = s.estimate_batch(G, T, pats, budgets, 13, **kw)
    host = s.estimate_batch(G, T, pats, budgets, 13, host_rounds=True, **kw)
    say(f"batch: {sum(r.converged for r in dev)}/32 converged, {sum(r.n for r in dev)} samples")
    for a, b in zip(dev, host):
        assert a.n == b.n and a.converged == b.converged and a.n_nonzero == b.n_nonzero
        assert abs(a.estimate - b.estimate) <= 1e-12 * abs(b.estimate)


@pytest.mark.parametrize("mode", ["switch", "always", "uniform"])
def test_time_to_eps_in_one_launch_equals_host_rounds(r20, mode):
    """The bench's time-to-+-1% runs (checks every 4,096 from 4,096, budget
    10^8) of the four headline patterns: same stop points and estimates on
    both paths."""
    g, s, G, T, O, TO = r20
    kw = dict(mode=mode, eps=0.01, delta=0.05, check_every=4096, min_samples=4096)
    for pid, name in enumerate(["5-clique", "5-cycle", "house", "4-star"]):
        p = synth.named_pattern(name)
        a = s.estimate(G, T, p, 10 ** 8, 17, pattern_id=pid, **kw)
        b = s.estimate(G, T, p, 10 ** 8, 17, pattern_id=pid, host_rounds=True, **kw)
        say(f"{name} {mode}: {a.n} samples, converged {bool(a.converged)}")
        assert a.n == b.n and a.converged == b.converged
        assert abs(a.estimate - b.estimate) <= 1e-12 * abs(b.estimate)
