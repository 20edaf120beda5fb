"""GPU: batched multi-pattern rounds, graph replay and launch-shape
invariance, through the C-ABI."""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.estimator import run_to_eps
from oracle.pattern import compile_pattern

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
def c1_state(sess):
    g = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    return g, G, T, oracle.Tables(g, cv_seed=1)


def _pats():
    named = [synth.named_pattern(n) for n in ("triangle", "4-cycle", "4-clique", "house", "5-cycle", "4-star")]
    rand = [p for p, _ in synth.random_pattern_set(10, seed=3, kmin=4, kmax=6)]
    return named + rand


def _same(a, b, rel=1e-9):
    assert a.n == b.n and a.n_nonzero == b.n_nonzero and a.converged == b.converged
    assert a.estimate == pytest.approx(b.estimate, rel=rel, abs=0.0)


@pytest.mark.parametrize("mode", ["switch", "uniform"])
def test_batch_equals_single_runs(sess, c1_state, mode):
    g, G, T, _ = c1_state
    pats = _pats()
    rng = np.random.Generator(np.random.PCG64(5))
    budgets = [int(x) for x in np.round(10 ** rng.uniform(3, 5.3, size=len(pats)))]
    say(f"batch exact budgets {mode}: {len(pats)} patterns, {sum(budgets)} samples")
    res = sess.estimate_batch(G, T, pats, budgets, 7, mode=mode, pattern_id=10)
    for i, (p, b) in enumerate(zip(pats, budgets)):
        single = sess.estimate(G, T, p, b, 7, mode=mode, pattern_id=10 + i)
        assert res[i].n == b
        _same(res[i], single)


def test_batch_run_to_eps_matches_single_and_oracle(sess, c1_state):
    g, G, T, OT = c1_state
    pats = [synth.named_pattern(n) for n in ("triangle", "4-cycle", "4-clique", "house")]
    budgets = [1 << 21] * len(pats)
    kw = dict(mode="switch", eps=0.02, delta=0.05, check_every=4096, min_samples=8192, pattern_id=3)
    say("batch run-to-eps")
    res = sess.estimate_batch(G, T, pats, budgets, 11, **kw)
    for i, p in enumerate(pats):
        single = sess.estimate(G, T, p, budgets[i], 11, **dict(kw, pattern_id=3 + i))
        _same(res[i], single)
        st, conv = run_to_eps(oracle.Sampler(g, OT, compile_pattern(p.k, p.edges), seed=11, pattern_id=3 + i),
                              0.02, 0.05, 4096, 8192, budgets[i])
        assert res[i].n == st.n and bool(res[i].converged) == conv
        assert res[i].estimate == pytest.approx(st.mean, rel=1e-9)


def test_graph_replay_equals_direct_launches(sess, c1_state):
    """Rounds replayed from the captured graph (many replays, with other
    work between them) give exactly what direct launches give."""
    g, G, T, _ = c1_state
    p = synth.named_pattern("house")
    kw = dict(mode="switch", eps=1e-9, check_every=5000, min_samples=0)
    say("graph replay vs direct")
    sess.set_launch(use_graphs=False)
    direct = sess.estimate(G, T, p, 200_000, 5, **kw)
    sess.set_launch(use_graphs=True)
    for rep in range(3):
        replay = sess.estimate(G, T, p, 200_000, 5, **kw)
        assert replay.n == direct.n == 200_000 and replay.sample_launches == 40
        assert replay.estimate == direct.estimate and replay.variance == direct.variance
        # unrelated work between replays
        other = sess.estimate(G, T, synth.named_pattern("triangle"), 10_000, rep, mode="uniform")
        assert other.n == 10_000


@pytest.mark.parametrize("shape", [(1, 1, 0), (2, 3, 0), (0, 16, 1), (0, 1, 2), (3, 0, 1), (0, 0, 2), (0, 0, 0, 1024),
                                   (0, 4, 1, 1 << 30)])
def test_launch_shape_invariance(sess, c1_state, shape):
    g, G, T, OT = c1_state
    p = synth.named_pattern("5-cycle")
    sess.set_launch(use_graphs=True)
    ref = sess.estimate(G, T, p, 300_000, 9)
    refrec = sess.dump(G, T, p, 9, np.arange(2000, dtype=np.uint64))
    say(f"launch shape {shape}")
    sess.set_launch(use_graphs=True, blocks_per_cu=shape[0], grab=shape[1], variant=shape[2],
                    hub_window=shape[3] if len(shape) > 3 else 0)
    got = sess.estimate(G, T, p, 300_000, 9)
    rec = sess.dump(G, T, p, 9, np.arange(2000, dtype=np.uint64))
    sess.set_launch(use_graphs=True)
    assert got.n == ref.n and got.estimate == ref.estimate and got.variance == ref.variance
    assert np.array_equal(rec.view(np.uint8), refrec.view(np.uint8))


def test_autotune_keeps_results(sess, c1_state):
    g, G, T, _ = c1_state
    pats = [synth.named_pattern(n) for n in ("house", "4-clique", "5-cycle")]
    ref = sess.estimate_batch(G, T, pats, [100_000] * 3, 4)
    say("autotune")
    tun = sess.autotune(G, T, pats, 20_000)
    assert tun.variant in (0, 1, 2) and tun.seconds > 0 and tun.seconds <= tun.default_seconds
    got = sess.estimate_batch(G, T, pats, [100_000] * 3, 4)
    sess.set_launch(use_graphs=True)
    for a, b in zip(ref, got):
        assert a.n == b.n and a.estimate == b.estimate


def test_batch_random_patterns_rmat_scale_small(sess):
    """The 32-pattern set on a small R-MAT graph: batch = single runs."""
    g = synth.rmat(14, 16, seed=14)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    pset = synth.random_pattern_set(32, seed=3)
    pats = [p for p, _ in pset]
    budgets = [max(1000, b // 20000) for _, b in pset]
    say(f"32-pattern batch on R-MAT-14, {sum(budgets)} samples")
    res = sess.estimate_batch(G, T, pats, budgets, 1, mode="switch")
    for i in (0, 5, 17, 31):
        single = sess.estimate(G, T, pats[i], budgets[i], 1, mode="switch", pattern_id=i)
        _same(res[i], single)
    assert all(r.n == b for r, b in zip(res, budgets))
    assert all(math.isfinite(r.estimate) for r in res)


@pytest.mark.parametrize("check", [2048, 1 << 14, 1 << 16])
def test_one_launch_run_to_eps_equals_host_rounds(sess, c1_state, check):
    """The persistent run to epsilon (checks, merges and stops on the device)
    stops every pattern at the same sample count as the round-by-round run
    with the checks on the host, with the same estimates; budgets that are
    not multiples of the reduction tile, and minimums between checks."""
    g, G, T, _ = c1_state
    pats = _pats()
    rng = np.random.Generator(np.random.PCG64(check))
    budgets = [int(x) for x in np.round(10 ** rng.uniform(3.5, 6.3, size=len(pats)))]
    kw = dict(mode="switch", eps=0.02, delta=0.05, check_every=check, min_samples=3 * check // 2)
    say(f"one launch vs rounds, check {check}")
    dev = sess.estimate_batch(G, T, pats, budgets, 21, **kw)
    host = sess.estimate_batch(G, T, pats, budgets, 21, host_rounds=True, **kw)
    assert any(r.converged for r in dev) and any(not r.converged for r in dev)
    for a, b, bud in zip(dev, host, budgets):
        _same(a, b, rel=1e-12)
        assert a.n <= bud
    for p, bud, a in list(zip(pats, budgets, dev))[:4]:
        single = sess.estimate(G, T, p, bud, 21, pattern_id=pats.index(p), **kw)
        _same(single, a, rel=1e-12)


def test_one_launch_batch_of_many_patterns_converges(sess, c1_state):
    """64 patterns at once, all to +-2%: every stop point equals the host
    rounds' (the window and ring hold 64 patterns)."""
    g, G, T, _ = c1_state
    pats = [p for p, _ in synth.random_pattern_set(58, seed=9, kmin=3, kmax=6)] + _pats()[:6]
    budgets = [1 << 22] * len(pats)
    kw = dict(mode="switch", eps=0.02, delta=0.05, check_every=4096, min_samples=4096)
    dev = sess.estimate_batch(G, T, pats, budgets, 5, **kw)
    host = sess.estimate_batch(G, T, pats, budgets, 5, host_rounds=True, **kw)
    for a, b in zip(dev, host):
        _same(a, b, rel=1e-12)


def test_batch_learned_equals_single_learned(sess, c1_state):
    """Learned tables per pattern in one batch (batch_learned) give each
    pattern the samples of its single learned estimate."""
    import torch
    g, G, T, OT = c1_state
    names = ["house", "5-cycle", "4-clique"]
    pats = [synth.named_pattern(n) for n in names]
    rng = np.random.Generator(np.random.PCG64(17))
    tabs_all, ptrs_all = [], []
    for p in pats:
        base = sess.step_log_weights(T, p).cpu().numpy()
        tabs = {}
        for i in sess.weighted_steps(p, "learned"):
            t = base[i].astype(np.int64) + rng.integers(-2 << 16, 2 << 16, size=base.shape[1])
            t = np.where(base[i] == np.iinfo(np.int32).min, np.iinfo(np.int32).min, t).astype(np.int32)
            tabs[i] = torch.from_numpy(t).to(sess.device)
        tabs_all.append(tabs)
        ptrs_all.append({i: tab.data_ptr() for i, tab in tabs.items()})
    arr = A.batch_learned_array(ptrs_all)
    budgets = [300_000, 200_000, 250_000]
    for eps in (0.0, 0.02):
        kw = dict(mode="learned", eps=eps, delta=0.05, check_every=1 << 14, min_samples=1 << 14)
        res = sess.estimate_batch(G, T, pats, budgets, 33, batch_learned=arr, **kw)
        for pid, (p, b, r) in enumerate(zip(pats, budgets, res)):
            single = sess.estimate(G, T, p, b, 33, learned=ptrs_all[pid], pattern_id=pid, **kw)
            _same(r, single, rel=1e-12)
    # and the samples are the oracle's
    idx = np.arange(2000, dtype=np.uint64)
    for pid, p in enumerate(pats):
        got = sess.dump(G, T, p, 33, idx, mode="learned", learned=ptrs_all[pid], pattern_id=pid)
        ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode="learned"), seed=33, pattern_id=pid,
                             learned={i: t.cpu().numpy() for i, t in tabs_all[pid].items()}).records(idx)
        for f in ("v", "num", "den", "x", "steps", "fail_step"):
            assert np.array_equal(got[f], ref[f]), (p.name, f)
