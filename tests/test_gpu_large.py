"""GPU: R-MAT scale 24 (16.7M vertices, ~5.2e8 CSR entries), generated on
the GPU, the graph of the batched and learned-proposal configurations.

Parity at full size: the oracle builds its own tables of the whole graph
from a host copy of the CSR (the OpenMP flavour, the same per-vertex
definitions) and replays sampled indices of the bench's four patterns, of
four patterns of the 32-pattern set and of a learned table set; records
must match element by element.  The estimator is also checked by
properties that hold at any size: the 4-star closed form and agreement of
the three proposal modes."""

import math
import sys

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
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_01388_amd.session import Session
    s = Session(0)
    say("generating R-MAT scale 24 on the GPU")
    off, nbr = synth.graphs.rmat_device(24, 16, seed=24, device=str(s.device))
    G = s.graph(off, nbr)
    T = s.tables(G, cv_seed=1)
    say(f"n={G.n} nnz={G.nnz}")
    yield s, G, T, off, nbr
    T.close()
    G.close()
    s.close()


@pytest.fixture(scope="module")
def big_oracle(big):
    """A host copy of the CSR and the oracle's own tables of every vertex."""
    import time
    s, G, T, off, nbr = big
    host = synth.CSR(off=off.cpu().numpy().view(np.uint64).copy(), nbr=nbr.cpu().numpy().view(np.uint32).copy())
    t0 = time.time()
    ot = oracle.Tables(host, cv_seed=1, threads=0)
    say(f"oracle tables of all {host.n} vertices in {time.time() - t0:.1f} s")
    return host, ot


def _compare_records(got, ref, what):
    for f in ("v", "num", "den", "x", "steps", "fail_step"):
        bad = np.flatnonzero(np.any((got[f] != ref[f]).reshape(len(got), -1), axis=1))
        assert bad.size == 0, (what, f, bad[:5])


def _indices(count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.unique(np.concatenate([np.arange(64), rng.integers(0, 1 << 40, count),
                                     [(1 << 32) - 1, 1 << 32, (1 << 63) + 5]]).astype(np.uint64))


def test_rmat24_full_tables_match_oracle(big, big_oracle):
    s, G, T, off, nbr = big
    host, ot = big_oracle
    got = T.export()
    for k in ("deg", "s2", "hits", "trials", "la", "lc"):
        bad = np.flatnonzero(got[k].astype(np.int64) != getattr(ot, k).astype(np.int64))
        assert bad.size == 0, (k, bad[:10])


@pytest.mark.parametrize("name,count", [("5-clique", 1500), ("5-cycle", 10000), ("house", 10000),
                                        ("4-star", 10000)])
def test_rmat24_records_parity_bench_patterns(big, big_oracle, name, count):
    """Sampled indices of the bench's patterns (switch mode, row tables on,
    as the bench's long runs use them) against the oracle."""
    s, G, T, off, nbr = big
    host, ot = big_oracle
    p = synth.named_pattern(name)
    idx = _indices(count, 240 + len(name))
    say(f"records of {idx.size} samples of {name} on scale 24")
    got = s.dump(G, T, p, 7, idx, mode="switch", rowtab="on")
    ref = oracle.Sampler(host, ot, compile_pattern(p.k, p.edges, mode="switch"), seed=7).records(idx, threads=0)
    _compare_records(got, ref, name)


@pytest.mark.parametrize("which", [0, 9, 17, 30])
def test_rmat24_records_parity_batch_patterns(big, big_oracle, which):
    """Four patterns of the seeded 32-pattern set, in a batch launch (pattern
    ids as the batch assigns them), against the oracle."""
    s, G, T, off, nbr = big
    host, ot = big_oracle
    p = synth.random_pattern_set(32, seed=3)[which][0]
    idx = _indices(2000, 300 + which)
    say(f"records of {idx.size} samples of batch pattern {which} (k={p.k}, {len(p.edges)} edges) on scale 24")
    got = s.dump(G, T, p, 13, idx, mode="switch", pattern_id=which)
    ref = oracle.Sampler(host, ot, compile_pattern(p.k, p.edges, mode="switch"), seed=13,
                         pattern_id=which).records(idx, threads=0)
    _compare_records(got, ref, which)


def test_rmat24_records_parity_learned(big, big_oracle):
    """A learned table set (BF16 inference of a network into Q16 tables, as
    a correction of f_approx) fed to both sides."""
    import torch
    from paper_2601_01388_amd.session import mlp_init
    s, G, T, off, nbr = big
    host, ot = big_oracle
    p = synth.named_pattern("house")
    feats = s.features(T)
    params = torch.from_numpy(mlp_init(5, 0.0, zero_output=False)).to(s.device)
    tabs = s.learned_tables(params, feats, p, base=s.step_log_weights(T, p))
    learned = {i: tab.data_ptr() for i, tab in tabs.items()}
    idx = _indices(4000, 77)
    say(f"records of {idx.size} learned samples of the house on scale 24")
    got = s.dump(G, T, p, 17, idx, mode="learned", learned=learned, rowtab="on")
    ref = oracle.Sampler(host, ot, compile_pattern(p.k, p.edges, mode="learned"), seed=17,
                         learned={i: tab.cpu().numpy() for i, tab in tabs.items()}).records(idx, threads=0)
    _compare_records(got, ref, "learned house")
    # the production estimate over a prefix equals the oracle's
    r = s.estimate(G, T, p, 1 << 14, 17, mode="learned", learned=learned)
    st, _ = oracle.Sampler(host, ot, compile_pattern(p.k, p.edges, mode="learned"), seed=17,
                           learned={i: tab.cpu().numpy() for i, tab in tabs.items()}).run_parallel(0, 1 << 14)
    assert abs(r.estimate - st.mean) <= 1e-9 * abs(st.mean)


def test_rmat24_tables_on_sampled_vertices(big):
    s, G, T, off, nbr = big
    host = synth.CSR(off=off.cpu().numpy().view(np.uint64), nbr=nbr.cpu().numpy().view(np.uint32))
    d = np.diff(host.off.astype(np.int64))
    rng = np.random.Generator(np.random.PCG64(24))
    vs = np.concatenate([rng.integers(0, host.n, 3000), np.argsort(d)[-200:], [0, host.n - 1]]).astype(np.uint64)
    say(f"tables of {vs.size} sampled vertices (the 200 largest degrees among them)")
    got = T.export()
    ref = oracle.tables_at(host, vs, cv_seed=1)
    for k in ("deg", "s2", "hits", "trials", "la", "lc"):
        assert np.array_equal(got[k][vs.astype(np.int64)], ref[k]), k


def test_rmat24_four_star_closed_form(big):
    s, G, T, off, nbr = big
    d = (off[1:] - off[:-1]).cpu().numpy().astype(np.float64)
    exact = 24.0 * float(np.sum(d * (d - 1) * (d - 2) * (d - 3) / 24.0))  # 4! * sum C(d, 4)
    p = synth.named_pattern("4-star")
    say("4-star on scale 24")
    r = s.estimate(G, T, p, 1 << 20, 5, mode="switch")
    se = math.sqrt(r.variance / r.n)
    assert abs(r.estimate - exact) <= 5 * se + 1e-9 * exact, (r.estimate, exact, se)
    assert abs(r.estimate / exact - 1) < 2e-3


def test_rmat24_modes_agree(big):
    s, G, T, off, nbr = big
    p = synth.named_pattern("5-cycle")
    res = {}
    for mode, n in (("switch", 1 << 22), ("always", 1 << 22), ("uniform", 1 << 23)):
        say(f"5-cycle {mode} on scale 24")
        res[mode] = s.estimate(G, T, p, n, 7, mode=mode)
    for a in res:
        for b in res:
            if a < b:
                ra, rb = res[a], res[b]
                se = math.sqrt(ra.variance / ra.n + rb.variance / rb.n)
                assert abs(ra.estimate - rb.estimate) <= 5 * se, (a, b, ra.estimate, rb.estimate, se)
