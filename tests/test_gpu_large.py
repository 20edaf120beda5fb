"""GPU: R-MAT scale 24 (16.7M vertices, ~5.2e8 CSR entries), generated on
the GPU.  The oracle cannot build the whole tables of this graph in test
time, so parity is checked on sampled vertices, and the estimator by
properties that hold at any size: the 4-star closed form and agreement of
the three proposal modes."""

import math
import sys

import numpy as np
import pytest

import oracle
import synth

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
