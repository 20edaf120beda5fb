"""GPU tests of the large-graph path: the counter-based R-MAT generator
(against its host twin), the blocked first-step table (against the oracle),
and a graph with more than 2^32 CSR slots (R-MAT scale 28, edge factor 16:
~8.6e9 slots, 34 GB of neighbours), where every slot index, offset and
first draw is a 64-bit quantity."""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle.pattern import compile_pattern
from synth import graphs

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


@pytest.mark.parametrize("scale,seed", [(10, 5), (13, 6)])
def test_generator_matches_host_twin(sess, scale, seed):
    off, nbr = graphs.rmat_gpu(scale, 16, seed=seed, device=str(sess.device), stage_bytes=1 << 24)
    host = graphs.rmat_counter(scale, 16, seed=seed)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), host.off)
    assert np.array_equal(nbr.cpu().numpy().view(np.uint32), host.nbr)


def test_generator_small_staging_splits_batches(sess):
    """A staging buffer far below the graph forces many sort and move
    batches; the graph is the same."""
    off, nbr = graphs.rmat_gpu(14, 16, seed=9, device=str(sess.device), stage_bytes=1 << 20)
    host = graphs.rmat_counter(14, 16, seed=9)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), host.off)
    assert np.array_equal(nbr.cpu().numpy().view(np.uint32), host.nbr)


@pytest.fixture(scope="module")
def c1g(sess):
    g = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    yield g, G, T, oracle.Tables(g, cv_seed=1)
    T.close()
    G.close()


@pytest.mark.parametrize("name", ["triangle", "4-clique", "house", "5-cycle", "4-star"])
@pytest.mark.parametrize("mode", ["switch", "always"])
def test_blocked_first_step_matches_oracle(sess, c1g, name, mode):
    g, G, T, OT = c1g
    p = synth.named_pattern(name)
    idx = np.concatenate([np.arange(3000), [(1 << 32) + 7, (1 << 63) + 1]]).astype(np.uint64)
    got = sess.dump(G, T, p, 7, idx, mode=mode, step1="blocks")
    ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode=mode), seed=7).records(idx)
    for f in ("v", "num", "den", "x", "steps", "fail_step"):
        assert np.array_equal(got[f], ref[f]), f
    a = sess.estimate(G, T, p, 1 << 18, 7, mode=mode, step1="blocks")
    b = sess.estimate(G, T, p, 1 << 18, 7, mode=mode, step1="full")
    assert a.estimate == b.estimate and a.variance == b.variance


def test_blocked_first_step_with_learned_table(sess, c1g):
    """A learned first-step table (the house's step 0 is weighted) read
    through the blocked path."""
    import torch
    g, G, T, OT = c1g
    p = synth.named_pattern("house")
    rng = np.random.Generator(np.random.PCG64(3))
    base = sess.step_log_weights(T, p).cpu().numpy()
    tabs = {}
    for i in sess.weighted_steps(p, "learned"):
        t = base[i].astype(np.int64) + rng.integers(-3 << 16, 3 << 16, size=base.shape[1])
        t = np.where(base[i] == np.iinfo(np.int32).min, np.iinfo(np.int32).min, t).astype(np.int32)
        tabs[i] = torch.from_numpy(t).to(sess.device)
    learned = {i: tab.data_ptr() for i, tab in tabs.items()}
    idx = np.arange(4000, dtype=np.uint64)
    got = sess.dump(G, T, p, 9, idx, mode="learned", learned=learned, step1="blocks")
    ref = oracle.Sampler(g, OT, compile_pattern(p.k, p.edges, mode="learned"), seed=9,
                         learned={i: tab.cpu().numpy() for i, tab in tabs.items()}).records(idx)
    for f in ("v", "num", "den", "x", "steps", "fail_step"):
        assert np.array_equal(got[f], ref[f]), f


@pytest.fixture(scope="module")
def r28(sess):
    import time
    import torch
    t0 = time.time()
    off, nbr = graphs.rmat_gpu(28, 16, seed=28, device=str(sess.device))
    torch.cuda.synchronize()
    say(f"R-MAT scale 28 generated in {time.time() - t0:.1f} s: nnz = {nbr.numel()}")
    assert nbr.numel() > (1 << 32)
    t0 = time.time()
    G = sess.graph(off, nbr, validate=True)
    torch.cuda.synchronize()
    say(f"loaded and validated in {time.time() - t0:.1f} s")
    t0 = time.time()
    T = sess.tables(G, cv_seed=1)
    torch.cuda.synchronize()
    say(f"tables in {time.time() - t0:.1f} s")
    yield off, nbr, G, T
    T.close()
    G.close()
    del off, nbr
    torch.cuda.empty_cache()


def test_rmat28_edge_uniform_first_draws_beyond_2_32(sess, r28):
    """The uniform first step draws a CSR slot r in [0, nnz) and takes its
    row: checked against a host binary search on the offsets, for draws on
    both sides of 2^32."""
    off, nbr, G, T = r28
    nnz = nbr.numel()
    host_off = off.cpu().numpy().view(np.uint64)
    idx = np.arange(20000, dtype=np.uint64)
    recs = sess.dump(G, T, synth.named_pattern("4-star"), 11, idx, mode="uniform")
    r = np.array([oracle.bounded(11, int(s) & 0xFFFFFFFF, int(s) >> 32, 0, 0, nnz) for s in idx], dtype=np.uint64)
    want = np.searchsorted(host_off, r, side="right") - 1
    high = r >= (1 << 32)
    say(f"{int(high.sum())} of {r.size} first draws at slots >= 2^32")
    assert high.sum() > 1000 and (~high).sum() > 1000
    assert np.array_equal(recs["v"][:, 0].astype(np.int64), want.astype(np.int64))
    d = np.diff(host_off.astype(np.int64))
    assert np.array_equal(recs["num"][:, 0], np.full(r.size, nnz, dtype=np.uint64))
    assert np.array_equal(recs["den"][:, 0].astype(np.int64), d[want])


def test_rmat28_four_star_closed_form(sess, r28):
    off, nbr, G, T = r28
    d = (off[1:] - off[:-1]).cpu().numpy().astype(np.float64)
    exact = float(np.sum(d * (d - 1) * (d - 2) * (d - 3)))  # 4! * sum C(d, 4)
    r = sess.estimate(G, T, synth.named_pattern("4-star"), 1 << 20, 5, mode="switch")
    se = math.sqrt(r.variance / r.n)
    say(f"4-star: {r.estimate:.6g} vs {exact:.6g} (se {se:.3g})")
    assert abs(r.estimate - exact) <= 5 * se + 1e-9 * exact


def test_rmat28_modes_agree(sess, r28):
    off, nbr, G, T = r28
    p = synth.named_pattern("5-cycle")
    res = {}
    for mode, n in (("switch", 1 << 21), ("always", 1 << 21), ("uniform", 1 << 22)):
        res[mode] = sess.estimate(G, T, p, n, 7, mode=mode)
        say(f"5-cycle {mode}: {res[mode].estimate:.6g} (rel se {math.sqrt(res[mode].variance / res[mode].n) / res[mode].estimate:.3g})")
    for a in res:
        for b in res:
            if a < b:
                ra, rb = res[a], res[b]
                se = math.sqrt(ra.variance / ra.n + rb.variance / rb.n)
                assert abs(ra.estimate - rb.estimate) <= 5 * se, (a, b, ra.estimate, rb.estimate, se)
