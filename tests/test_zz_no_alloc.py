"""GPU: agis_estimate_noalloc (the entry point for callers that cannot
allocate device memory) against agis_estimate, through the C-ABI: two calls
in a row, the second with a smaller input, fixed-count and run-to-eps; no
device memory is taken by a call; inputs beyond the fixed workspace are
refused with a clear error."""

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


def _noalloc(sess, G, T, p, n, seed, **kw):
    return A.agis_estimate_noalloc(sess.ctx, G.handle, T.handle, A.make_pattern(p.k, p.adj8()), n, seed,
                                   A.make_params(**kw))


def _same(a, b, what):
    assert a.n == b.n, (what, a.n, b.n)
    assert a.converged == b.converged, what
    assert abs(a.estimate - b.estimate) <= 1e-9 * abs(b.estimate), (what, a.estimate, b.estimate)
    assert abs(a.variance - b.variance) <= 1e-9 * abs(b.variance), (what, a.variance, b.variance)
    assert a.n_nonzero == b.n_nonzero, what


def test_two_calls_in_a_row_match_the_allocating_entry_point(sess):
    big = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    small = synth.chung_lu(n=2_000, m=12_000, gamma=2.1, seed=4)
    cases = [(big, "4-clique", 3 << 20, "switch"), (small, "house", 1 << 16, "always")]
    for g, name, n, mode in cases:
        G = sess.graph(g.off, g.nbr)
        T = sess.tables(G, cv_seed=1)
        p = synth.named_pattern(name)
        say(f"noalloc {name} {mode} n={n} on a graph of {g.n} vertices")
        got = _noalloc(sess, G, T, p, n, 7, mode=mode, pattern_id=3)
        ref = sess.estimate(G, T, p, n, 7, mode=mode, pattern_id=3)
        assert got.status == A.AGIS_OK
        _same(got, ref, (name, mode))
        T.close()
        G.close()


def test_run_to_eps_stops_where_the_allocating_entry_point_stops(sess):
    g = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    for name, n in (("triangle", 1 << 22), ("4-cycle", 1 << 18)):
        p = synth.named_pattern(name)
        kw = dict(mode="switch", eps=0.01, delta=0.05, check_every=1 << 14, min_samples=1 << 14)
        got = _noalloc(sess, G, T, p, n, 11, **kw)
        ref = sess.estimate(G, T, p, n, 11, **kw)
        say(f"to eps {name}: n={got.n} status {got.status}")
        assert got.status == ref.status
        _same(got, ref, name)
    T.close()
    G.close()


def test_a_call_takes_no_device_memory(sess):
    import torch
    g = synth.rmat(16, 16, seed=16)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    p = synth.named_pattern("5-cycle")
    first = _noalloc(sess, G, T, p, 1 << 18, 5, mode="switch")  # loads the code objects
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    again = _noalloc(sess, G, T, p, 1 << 18, 5, mode="switch")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    _same(again, first, "repeat")
    ref = sess.estimate(G, T, p, 1 << 18, 5, mode="switch")
    _same(again, ref, "vs allocating")
    T.close()
    G.close()


def test_inputs_beyond_the_workspace_are_refused(sess):
    # a star whose centre has 2^23 neighbours: one workgroup's scratch
    # (4 waves x 2 x (2^23 + 1) x 4 bytes) exceeds the 256 MiB workspace
    leaves = 1 << 23
    off = np.zeros(leaves + 2, dtype=np.uint64)
    off[1] = leaves
    off[2:] = leaves + np.arange(1, leaves + 1, dtype=np.uint64)
    nbr = np.concatenate([np.arange(1, leaves + 1, dtype=np.uint32), np.zeros(leaves, dtype=np.uint32)])
    G = sess.graph(off, nbr, validate=False)
    T = sess.tables(G, cv_seed=1)
    p = synth.named_pattern("4-star")
    with pytest.raises(A.AgisError) as e:
        _noalloc(sess, G, T, p, 1 << 10, 1, mode="switch", wave_samples=True)
    assert e.value.code == A.AGIS_E_UNSUPPORTED
    say(f"refused: {e.value}")
    assert "workspace" in str(e.value)
    # the allocating entry point still serves it
    r = sess.estimate(G, T, p, 1 << 10, 1, mode="switch", wave_samples=True)
    assert r.n == 1 << 10
    # the lane sampler (which stars run on by default) keeps no candidate
    # set, so it needs no scratch and the fixed workspace serves the star
    a = _noalloc(sess, G, T, p, 1 << 10, 1, mode="switch")
    _same(a, r, "lanes in the fixed workspace")
    T.close()
    G.close()
