"""GPU parity of the lane sampler (one sample per lane) for plans whose
steps after the first are uniform draws from one matched vertex's row:
stars under switching, every tree under f_uniform.  Its records equal the
oracle's and the wave sampler's, bit for bit, and so do its estimates."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.pattern import compile_pattern

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2601_01388_amd")

SEED = 7


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
    g = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    yield g, G, T, oracle.Tables(g, cv_seed=1)
    T.close()
    G.close()


def _indices(m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    far = rng.integers(0, 1 << 62, size=m // 4, dtype=np.uint64)
    edge = np.array([(1 << 32) - 1, 1 << 32, (1 << 63) - 1, (1 << 64) - 1], dtype=np.uint64)
    return np.concatenate([np.arange(m, dtype=np.uint64), far, edge])


def _same_records(a, b, label):
    for f in ("v", "num", "den", "x", "steps", "fail_step"):
        assert np.array_equal(a[f], b[f]), (label, f)


def _random_tree(k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(int(rng.integers(0, i)), i) for i in range(1, k)]


# (name, pattern, modes under which every later step is a uniform one-row draw)
LANE_CASES = [("edge", synth.named_pattern("edge"), ["uniform", "switch", "always"])]
LANE_CASES += [(f"{l}-star", synth.patterns.star(l), ["uniform", "switch", "always"]) for l in range(2, 8)]
LANE_CASES += [(f"{k}-path", synth.patterns.path(k), ["uniform"]) for k in range(3, 9)]
LANE_CASES += [(f"tree{k}.{s}", synth.patterns._mk(k, _random_tree(k, s), f"tree{k}"), ["uniform"])
               for k, s in ((5, 1), (6, 2), (7, 3), (8, 4))]


@pytest.mark.parametrize("name,pat,modes", LANE_CASES, ids=[c[0] for c in LANE_CASES])
def test_lane_records_equal_oracle_and_wave(sess, c1, name, pat, modes):
    g, G, T, OT = c1
    idx = _indices(2500, seed=len(name) * 31 + pat.k)
    for mode in modes:
        say(f"lane records {name} {mode}")
        lanes = sess.dump(G, T, pat, SEED, idx, mode=mode, pattern_id=3)
        wave = sess.dump(G, T, pat, SEED, idx, mode=mode, pattern_id=3, wave_samples=True)
        ref = oracle.Sampler(g, OT, compile_pattern(pat.k, pat.edges, mode=mode), seed=SEED,
                             pattern_id=3).records(idx)
        _same_records(lanes, ref, f"{name}/{mode} lanes vs oracle")
        _same_records(wave, ref, f"{name}/{mode} wave vs oracle")


def test_lane_failing_steps(sess):
    """Rows too short for the pattern: stars on a ring and on a path graph
    fail at the step whose row has no unmatched vertex left; the graph
    without edges fails at step 0."""
    for gname, g in (("ring", synth.ring_graph(40)), ("path", synth.csr_from_edges(
            30, list(range(29)), list(range(1, 30)))), ("empty", synth.csr_from_edges(5, [], []))):
        G = sess.graph(g.off, g.nbr)
        T = sess.tables(G)
        OT = oracle.Tables(g)
        idx = np.arange(700, dtype=np.uint64)
        for leaves in (2, 3, 5):
            p = synth.patterns.star(leaves)
            for mode in ("uniform", "switch"):
                got = sess.dump(G, T, p, 5, idx, mode=mode)
                ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode=mode), seed=5).records(idx)
                _same_records(got, ref, f"{gname}/{leaves}-star/{mode}")
                if leaves >= 3:  # no vertex has three neighbours
                    assert np.all(ref["fail_step"] >= 0)
                r = sess.estimate(G, T, p, 5000, 5, mode=mode)
                w = sess.estimate(G, T, p, 5000, 5, mode=mode, wave_samples=True)
                assert r.estimate == w.estimate and r.n_nonzero == w.n_nonzero
        T.close()
        G.close()


@pytest.mark.parametrize("mode", ["switch", "uniform"])
def test_lane_estimates_equal_wave_estimates(sess, c1, mode):
    """Same weights in the same slots, so the same reduction: the estimates
    agree exactly, for single runs, ragged sizes and batches of lane plans."""
    g, G, T, OT = c1
    pats = [synth.patterns.star(3), synth.patterns.star(4), synth.patterns.star(6)]
    if mode == "uniform":
        pats += [synth.patterns.path(5), synth.patterns.path(8)]
    for n in (1, 63, 2049, 300_001):
        for pid, p in enumerate(pats):
            a = sess.estimate(G, T, p, n, 11, mode=mode, pattern_id=pid)
            b = sess.estimate(G, T, p, n, 11, mode=mode, pattern_id=pid, wave_samples=True)
            assert a.estimate == b.estimate and a.variance == b.variance and a.n == b.n, (p.name, n)
    budgets = [70_000 + 9_999 * i for i in range(len(pats))]
    a = sess.estimate_batch(G, T, pats, budgets, 13, mode=mode)
    b = sess.estimate_batch(G, T, pats, budgets, 13, mode=mode, wave_samples=True)
    for ra, rb in zip(a, b):
        assert ra.estimate == rb.estimate and ra.variance == rb.variance and ra.n == rb.n
    # a batch with one plan the lane sampler does not serve runs on waves
    mixed = pats + [synth.named_pattern("triangle")]
    c = sess.estimate_batch(G, T, mixed, budgets + [50_000], 13, mode=mode)
    for ra, rc in zip(a, c):
        assert ra.estimate == rc.estimate and ra.variance == rc.variance


def test_lane_launch_shapes_and_graph_replay(sess, c1):
    """Grabs of 1 to 8 (64 slots each), fewer workgroups, direct launches
    and graph replays: the same estimate."""
    g, G, T, OT = c1
    p = synth.patterns.star(4)
    ref = sess.estimate(G, T, p, 1 << 20, 3, mode="switch")
    try:
        for graphs, blocks, grab in ((1, 0, 1), (1, 1, 8), (0, 2, 2), (0, 0, 4), (1, 0, 3)):
            sess.set_launch(use_graphs=graphs, blocks_per_cu=blocks, grab=grab, variant=0, hub_window=0)
            for _ in range(2):
                r = sess.estimate(G, T, p, 1 << 20, 3, mode="switch")
                assert r.estimate == ref.estimate and r.variance == ref.variance, (graphs, blocks, grab)
    finally:
        sess.set_launch(use_graphs=1, blocks_per_cu=0, grab=0, variant=0, hub_window=0)


def test_lane_meter_runs_its_own_kernel(sess, c1):
    """The metered requests of the lane sampler (per-lane binary searches)
    differ from the wave sampler's (64-lane probes) while the weights agree:
    both samplers ran."""
    g, G, T, OT = c1
    p = synth.patterns.star(4)
    idx = np.arange(4096, dtype=np.uint64)
    a = sess.meter(G, T, p, 5, idx, mode="switch")
    b = sess.meter(G, T, p, 5, idx, mode="switch", wave_samples=True)
    # columns: read bytes, written bytes, segments, requests
    assert np.all(a[:, 1] == 8) and np.all(b[:, 1] == 8)
    assert np.all(a[:, 0] > 0) and np.all(a[:, 2] > 0)
    assert not np.array_equal(a[:, 0], b[:, 0])


def test_lane_sampler_at_rmat_scale_20(sess):
    """The bench graph: the 4-star's records on sampled indices against the
    oracle (its own tables from the host CSR), and its estimate against
    4! x sum C(d, 4)."""
    import math
    g = synth.rmat(20, 16, seed=20)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    OT = oracle.Tables(g, cv_seed=1, threads=8)
    p = synth.named_pattern("4-star")
    idx = _indices(4000, seed=20)
    got = sess.dump(G, T, p, 7, idx, mode="switch")
    ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode="switch"), seed=7).records(idx)
    _same_records(got, ref, "rmat20 4-star")
    d = np.diff(g.off).astype(np.int64)
    exact = float(sum(math.perm(int(x), 4) for x in d[d >= 4]))
    r = sess.estimate(G, T, p, 1 << 24, 5, mode="switch")
    se = math.sqrt(r.variance / r.n)
    say(f"rmat20 4-star lanes: {r.estimate:.8g} vs {exact:.8g} (se {se:.3g})")
    assert abs(r.estimate - exact) <= 5 * se + 1e-9 * exact
    T.close()
    G.close()
