"""GPU tests of the proposal-table cache: the f_approx tables an estimate
builds (step weights, row pick tables, the first-step table) are kept with
the graph's tables and reused by later calls of the same step signature;
results never depend on whether a table came from the cache."""

import sys

import numpy as np
import pytest

import synth

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


@pytest.fixture(scope="module")
def c1(sess):
    g = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    G = sess.graph(g.off, g.nbr)
    yield g, G
    G.close()


def _same(a, b):
    assert a.n == b.n and a.estimate == b.estimate and a.variance == b.variance


def test_cached_tables_give_the_fresh_results(sess, c1):
    """Every call on one tables handle (so from the second on, from the
    cache) equals the first call on a fresh handle, across patterns, modes,
    term sets, first-step layouts and row tables on and off, in any order."""
    g, G = c1
    cases = []
    for name in ("house", "5-cycle", "4-clique", "diamond", "4-path"):
        for mode in ("switch", "always"):
            for terms in ("all", "f1"):
                for step1 in ("full", "blocks"):
                    cases.append((name, dict(mode=mode, terms=terms, step1=step1, rowtab="on")))
    cases.append(("house", dict(mode="switch", rowtab="off")))
    T = sess.tables(G, cv_seed=1)
    first = {}
    rng = np.random.Generator(np.random.PCG64(5))
    for rep in range(2):
        order = rng.permutation(len(cases))
        for c in order:
            name, kw = cases[c]
            r = sess.estimate(G, T, synth.named_pattern(name), 200_000, 9, **kw)
            key = (name, tuple(sorted(kw.items())))
            if key in first:
                _same(r, first[key])
            else:
                first[key] = r
    # a fresh handle (empty cache) agrees with the cached results
    T2 = sess.tables(G, cv_seed=1)
    for (name, kwt), r in list(first.items())[::7]:
        _same(sess.estimate(G, T2, synth.named_pattern(name), 200_000, 9, **dict(kwt)), r)
    # records through cached tables equal those of a fresh handle
    idx = np.arange(3000, dtype=np.uint64)
    for name in ("house", "4-clique"):
        a = sess.dump(G, T, synth.named_pattern(name), 3, idx, rowtab="on")
        T3 = sess.tables(G, cv_seed=1)
        b = sess.dump(G, T3, synth.named_pattern(name), 3, idx, rowtab="on")
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
        T3.close()
    # a batch whose patterns share signatures, twice
    pats = [synth.named_pattern(n) for n in ("house", "5-cycle", "4-clique", "diamond", "6-cycle")]
    x = sess.estimate_batch(G, T, pats, [150_000] * 5, 4)
    y = sess.estimate_batch(G, T, pats, [150_000] * 5, 4)
    z = sess.estimate_batch(G, T2, pats, [150_000] * 5, 4)
    for a, b, c in zip(x, y, z):
        _same(a, b)
        _same(a, c)
    T2.close()
    T.close()


def test_learned_tables_are_read_at_every_call(sess, c1):
    """Tables built from a caller's learned weights are not kept: changing
    the weights in place (same device pointer) changes the next estimate,
    which equals a fresh handle's estimate with the new weights."""
    import torch
    g, G = c1
    T = sess.tables(G, cv_seed=1)
    p = synth.named_pattern("house")
    base = sess.step_log_weights(T, p)
    steps = sess.weighted_steps(p, "learned")
    tabs = {i: base[i].clone() for i in steps}
    ptrs = {i: t.data_ptr() for i, t in tabs.items()}
    a = sess.estimate(G, T, p, 300_000, 5, mode="learned", learned=ptrs, rowtab="on")
    rng = np.random.Generator(np.random.PCG64(1))
    for i, t in tabs.items():
        noise = torch.from_numpy(rng.integers(-4 << 16, 4 << 16, size=t.numel()).astype(np.int32)).to(t.device)
        keep = t != torch.iinfo(torch.int32).min
        t.copy_(torch.where(keep, t + noise, t))
    torch.cuda.synchronize()
    b = sess.estimate(G, T, p, 300_000, 5, mode="learned", learned=ptrs, rowtab="on")
    T2 = sess.tables(G, cv_seed=1)
    c = sess.estimate(G, T2, p, 300_000, 5, mode="learned", learned=ptrs, rowtab="on")
    assert a.variance != b.variance
    _same(b, c)
    T2.close()
    T.close()


def test_cache_keeps_the_per_estimate_table_time_down(sess, c1):
    """The second estimate of a signature builds no table: its table time is
    below the first's (which builds the first-step, step-weight and row
    tables)."""
    g, G = c1
    T = sess.tables(G, cv_seed=1)
    p = synth.named_pattern("house")
    a = sess.estimate(G, T, p, 100_000, 1, rowtab="on")
    b = sess.estimate(G, T, p, 100_000, 1, rowtab="on")
    say(f"table seconds: first {a.tables_seconds:.6f}, cached {b.tables_seconds:.6f}")
    assert b.tables_seconds < a.tables_seconds
    T.close()


def test_release_scratch_gives_memory_back_with_the_same_results(sess, c1):
    """agis_release_scratch frees the sampler's kept buffers (the free device
    memory grows by at least the waves' scratch) and later estimates, fixed
    budgets and runs to eps alike, equal those before it."""
    import torch
    g, G = c1
    T = sess.tables(G, cv_seed=1)
    p = synth.named_pattern("house")
    a = sess.estimate(G, T, p, 300_000, 3)
    e = sess.estimate(G, T, p, 1 << 24, 4, eps=0.02, check_every=1 << 13, min_samples=1 << 13)
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    sess.release_scratch()
    sess.release_scratch()  # nothing left to free: still fine
    after = torch.cuda.mem_get_info()[0]
    # a wave's scratch is two arrays of (max degree + 1) entries
    per_wave = 2 * 4 * (int(np.diff(g.off).max()) + 1)
    say(f"released {(after - before) / 2 ** 20:.1f} MiB (one wave's scratch {per_wave / 1024:.1f} KiB)")
    assert after - before >= 256 * per_wave
    _same(sess.estimate(G, T, p, 300_000, 3), a)
    e2 = sess.estimate(G, T, p, 1 << 24, 4, eps=0.02, check_every=1 << 13, min_samples=1 << 13)
    _same(e2, e)
    assert e2.converged == e.converged
    T.close()
