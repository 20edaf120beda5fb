"""GPU tests of the measurement and run-control entry points: request
metering of the sampler (agis_meter_samples), the random-gather ceiling
(agis_gather_bench), resuming a run at a sample index
(agis_run_params.first_sample) and cancelling a run between rounds
(agis_run_params.cancel).  Everything goes through the C-ABI."""

import ctypes
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import synth
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
def c1g(sess):
    g = synth.chung_lu(n=10_000, m=100_000, gamma=2.1, seed=1)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1)
    yield g, G, T
    T.close()
    G.close()


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "4-clique", "house", "4-star"])
def test_meter_is_a_pure_function_of_the_sample(sess, c1g, name):
    """The request counts of a sample depend only on the sample (its path),
    not on the launch shape or on which other samples share the launch."""
    g, G, T = c1g
    p = synth.named_pattern(name)
    idx = np.arange(0, 3000, dtype=np.uint64) * 7919
    say(f"meter {name}")
    a = sess.meter(G, T, p, 7, idx, mode="switch", rowtab="on")
    sess.set_launch(False, 1, 1, 0, 0)
    b = sess.meter(G, T, p, 7, idx[::-1].copy(), mode="switch", rowtab="on")[::-1]
    sess.set_launch(True, 0, 0, 0, 0)
    assert np.array_equal(a, b)
    rb, wb, segs, reqs = a[:, 0], a[:, 1], a[:, 2], a[:, 3]
    # every sample reads its first-step entry and writes its weight slot
    assert (rb >= 8).all() and (wb >= 8).all()
    assert (segs >= 2).all() and (reqs >= 2).all()
    # a segment holds at most 64 bytes of one access, and a request at most
    # 64 lanes x 16 bytes
    assert (rb + wb <= 64 * segs + 64 * reqs).all()
    assert (rb + wb <= 1024 * reqs).all()


def test_meter_counts_a_star_exactly(sess, c1g):
    """On the 4-star every step after the first is an O(1) draw from the
    centre's row; the counts then follow from the record: step 0 (guide 8 B,
    the prefix search, the weight 4 B), then per later step the row offsets
    16 B, the search probes for the matched leaves, the drawn neighbour 4 B
    (not at the last step, which only counts), and the weight slot 8 B."""
    g, G, T = c1g
    p = synth.named_pattern("4-star")
    idx = np.arange(2000, dtype=np.uint64)
    recs = sess.dump(G, T, p, 7, idx, mode="switch", rowtab="on")
    ok = recs["fail_step"] < 0
    assert ok.any()
    # steps 1..4: 16 B offsets each, drawn neighbours at steps 1..3, 8 B slot
    fixed = 4 * 16 + 3 * 4
    # the wave sampler: at least one 64-lane probe of the prefix
    m = sess.meter(G, T, p, 7, idx, mode="switch", rowtab="on", wave_samples=True)
    assert (m[ok, 0] >= 8 + 4 + 8 * 1 + fixed).all()
    assert (m[ok, 1] == 8).all()  # only the weight slot is written
    # the lane sampler (the default for stars): the leaves are drawn from
    # the centre's row, so their positions are known and nothing is
    # searched after step 0; step 0 reads the guide, 8 B per probe of its
    # binary search between the guide's bounds (at most log2 n + 1), and
    # the weight
    m = sess.meter(G, T, p, 7, idx, mode="switch", rowtab="on")
    probes = (m[ok, 0].astype(np.int64) - (8 + 4 + fixed))
    assert (probes >= 0).all() and (probes % 8 == 0).all()
    assert (probes // 8 <= int(np.log2(g.n)) + 1).all()
    assert (m[ok, 1] == 8).all()


@pytest.mark.parametrize("seg", [4, 16, 64, 256, 1024])
def test_gather_bench_rates(sess, seg):
    import torch
    buf = torch.arange(1 << 26, dtype=torch.int64, device=sess.device)  # 512 MiB
    say(f"gather {seg}")
    dep = sess.gather_bench(buf, seg, True, waves_per_cu=28, rounds=64)
    ind = sess.gather_bench(buf, seg, False, waves_per_cu=28, rounds=64)
    for sec, ub in (dep, ind):
        assert sec > 0 and np.isfinite(sec)
        assert ub > 0 and ub % (64 * 64 * (16 if seg >= 16 else seg)) == 0
    # independent reads keep more in flight than a dependent chain
    assert ind[1] / ind[0] > 0.5 * dep[1] / dep[0]


def test_gather_bench_rejects_bad_arguments(sess):
    import torch
    buf = torch.zeros(1 << 20, dtype=torch.int64, device=sess.device)
    sink = torch.zeros(1024, dtype=torch.int64, device=sess.device)
    for seg, wpc, rounds in ((3, 28, 8), (2048, 28, 8), (64, 30, 8), (64, 28, 0)):
        with pytest.raises(A.AgisError):
            A.agis_gather_bench(sess.ctx, buf.data_ptr(), buf.numel() * 8, seg, False, wpc, rounds, 1,
                                sink.data_ptr())


@pytest.mark.parametrize("name", ["triangle", "house"])
def test_resume_continues_the_sample_sequence(sess, c1g, name):
    """A run over [N, 2N) (first_sample = N) equals the oracle over the same
    indices, and the two halves merge into the run over [0, 2N)."""
    g, G, T = c1g
    p = synth.named_pattern(name)
    N = 1 << 16
    r0 = sess.estimate(G, T, p, N, 7, mode="switch")
    r1 = sess.estimate(G, T, p, N, 7, mode="switch", first_sample=N)
    rall = sess.estimate(G, T, p, 2 * N, 7, mode="switch")
    ot = oracle.Tables(g, cv_seed=1)
    st, _, _ = oracle.Sampler(g, ot, compile_pattern(p.k, p.edges, mode="switch"), seed=7).run(N, N)
    assert r1.n == N
    assert abs(r1.estimate - st.mean) <= 1e-9 * abs(st.mean)
    mean = (r0.estimate + r1.estimate) / 2
    assert abs(mean - rall.estimate) <= 1e-9 * abs(rall.estimate)
    # records at the resumed indices are the oracle's
    idx = np.arange(N, N + 512, dtype=np.uint64)
    got = sess.dump(G, T, p, 7, idx, mode="switch")
    ref = oracle.Sampler(g, ot, compile_pattern(p.k, p.edges, mode="switch"), seed=7).records(idx)
    for f in ("v", "num", "den", "x", "steps", "fail_step"):
        assert np.array_equal(got[f], ref[f]), f


def test_cancel_before_start_returns_empty_partial(sess, c1g):
    g, G, T = c1g
    flag = ctypes.c_int32(1)
    r = sess.estimate(G, T, synth.named_pattern("triangle"), 1 << 20, 7, mode="switch", cancel=flag)
    assert r.status == A.AGIS_E_CANCELLED
    assert r.n == 0


def test_cancel_mid_run_keeps_a_consistent_prefix(sess, c1g):
    """A flag raised while a long run-to-eps is in flight stops it; the
    partial result is the estimate of a prefix of the sample sequence made
    of whole reduction tiles of 2048 (the same as a fixed run of that many
    samples), in the one-launch run and in the round-by-round run."""
    g, G, T = c1g
    p = synth.named_pattern("4-clique")
    flag = ctypes.c_int32(0)

    def raise_flag():
        time.sleep(0.3)
        flag.value = 1

    for host_rounds in (False, True):
        flag.value = 0
        th = threading.Thread(target=raise_flag)
        th.start()
        # eps far below reach: only the flag (or the large budget) ends the run
        budget = 1 << 32
        r = sess.estimate(G, T, p, budget, 7, mode="uniform", eps=1e-9, delta=0.05, check_every=1 << 16,
                          min_samples=1 << 16, cancel=flag, host_rounds=host_rounds)
        th.join()
        say(f"cancelled after {r.n} samples (host rounds {host_rounds})")
        assert r.status == A.AGIS_E_CANCELLED
        assert 0 < r.n < budget and r.n % 2048 == 0
        ref = sess.estimate(G, T, p, r.n, 7, mode="uniform")
        assert abs(r.estimate - ref.estimate) <= 1e-9 * abs(ref.estimate)
