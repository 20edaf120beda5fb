"""Pins of the learned-proposal oracle (FP64 network, features, targets)."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import judges, mlp
from oracle.pattern import compile_pattern


def test_gelu_identities():
    a = np.linspace(-6, 6, 101)
    # Phi(a) + Phi(-a) = 1  =>  gelu(a) - gelu(-a) = a
    assert np.allclose(mlp.gelu(a) - mlp.gelu(-a), a, atol=1e-14)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5
    assert np.allclose(mlp.gelu(np.array([10.0])), 10.0)
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(a), (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def _random_problem(seed, rows=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.normal(0, 0.3, size=mlp.N_PARAMS)
    feats = rng.uniform(0, 12, size=(30, 4))
    vtx = rng.integers(0, 30, size=rows)
    cls = rng.integers(0, 5, size=rows)
    x = mlp.inputs(feats, vtx, cls)
    target = rng.uniform(0, 20, size=rows)
    weight = rng.integers(1, 9, size=rows).astype(np.float64)
    return theta, x, target, weight


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    theta, x, t, w = _random_problem(seed)
    ws = w.sum()
    g = mlp.grad(theta, x, t, w, ws)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1, 0, 520, 4700]])
    for p in idx:
        h = 1e-5 * max(1.0, abs(theta[p]))
        tp = theta.copy(); tp[p] += h
        tm = theta.copy(); tm[p] -= h
        fd = (mlp.loss(tp, x, t, w, ws) - mlp.loss(tm, x, t, w, ws)) / (2 * h)
        assert fd == pytest.approx(g[p], rel=1e-6, abs=1e-8), p


def test_inputs_one_hot_positions():
    feats = np.arange(12, dtype=np.float64).reshape(3, 4)
    x = mlp.inputs(feats, [2, 0, 1, 1], [0, 1, 2, 7])
    assert np.array_equal(x[:, :4], feats[[2, 0, 1, 1]])
    assert np.array_equal(x[:, 4:], np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]]))


def test_h_index_definition():
    assert mlp.h_index([5, 3, 3, 1]) == 3
    assert mlp.h_index([]) == 0
    assert mlp.h_index([1, 1, 1]) == 1
    assert mlp.h_index([10, 9, 8, 7, 6]) == 5
    # K_n: every neighbour has degree n - 1
    k6 = synth.complete_graph(6)
    t = oracle.Tables(k6, exact_cv=True)
    f = mlp.features(k6, t)
    assert np.allclose(f[:, 3], math.log2(1 + 5))
    assert np.allclose(f[:, 2], math.log2(1 + 10))  # C_v = 1: C(5, 2) triangles at each vertex
    # star: centre sees leaves of degree 1 (h = 1); leaves see the centre (h = 1)
    st = synth.star_graph(5)
    f = mlp.features(st, oracle.Tables(st))
    assert np.allclose(f[:, 3], 1.0) and f[0, 0] == math.log2(6)


def _record_of(tau, s, k):
    """num/den of a trajectory from the sampler's own step distributions."""
    rec = {"v": np.zeros(8, dtype=np.uint32), "num": np.zeros(8, dtype=np.uint64), "den": np.zeros(8, dtype=np.uint64)}
    for i, v in enumerate(tau):
        vv, ww = s.step_distribution(i, list(tau[:i]))
        w = dict(zip(vv.tolist(), ww.tolist()))
        rec["v"][i] = v
        rec["num"][i] = sum(w.values())
        rec["den"][i] = w[v]
    return rec


@pytest.mark.parametrize("name", ["house", "4-clique", "5-cycle"])
def test_targets_are_unbiased_extension_counts(name):
    """Over the whole sampling tree, E[R_i ; v_i = v] = P(v_i = v) n_(.., v):
    for step 0 that is P(v_1 = v) times the number of embeddings mapping the
    first pattern vertex to v (Theorem 2 applied to the remaining steps)."""
    g = synth.graphs.skewed_tiny_graph(9, seed=3)
    p = synth.named_pattern(name)
    c = compile_pattern(p.k, p.edges, mode="switch")
    s = oracle.Sampler(g, oracle.Tables(g, cv_seed=2), c, seed=1)
    k = p.k
    expect = np.zeros(g.n, dtype=object)
    got = np.zeros(g.n, dtype=object)
    prob0 = np.zeros(g.n, dtype=object)

    def walk(i, tau, prob):
        if i == k:
            rec = _record_of(tau, s, k)
            rec["steps"], rec["fail_step"] = k, -1
            sums, _ = mlp.targets_from_records([rec], k, g.n)
            got[tau[0]] += prob * Fraction(sums[0, tau[0]])
            return
        vv, ww = s.step_distribution(i, tau)
        tot = int(ww.sum())
        if tot == 0:
            return  # failed branch: contributes R = 0
        for v, w in zip(vv.tolist(), ww.tolist()):
            if w:
                pr = prob * Fraction(int(w), tot)
                if i == 0:
                    prob0[v] += pr
                walk(i + 1, tau + [v], pr)

    walk(0, [], Fraction(1))
    # brute-force embeddings per image of the first matched pattern vertex
    first = c["order"][0]
    adj = g.adjacency_sets()
    import itertools
    per = np.zeros(g.n, dtype=np.int64)
    for m in itertools.permutations(range(g.n), k):
        if all(m[b] in adj[m[a]] for a, b in p.edges):
            per[m[first]] += 1
    for v in range(g.n):
        expect[v] = prob0[v] * per[v]
        assert abs(float(got[v]) - float(expect[v])) <= 1e-9 * max(1.0, float(expect[v])), (v, got[v], expect[v])
