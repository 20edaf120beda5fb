"""GPU: divergence of the first-step proposals the library samples from
(f_uniform, the incremental versions of f_approx, learned) from the ideal
first-step distribution given by exact rooted counts (the oracle's
backtracking judge), as in the paper's analysis of the approximation."""

import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import judges
from oracle.pattern import compile_pattern

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2601_01388_amd")


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def _kl(ideal, q, total):
    p = ideal.astype(np.float64) / ideal.sum()
    f = q.astype(np.float64) / float(total)
    m = p > 0
    assert np.all(f[m] > 0)
    return float(np.sum(p[m] * np.log(p[m] / f[m])))


def test_first_step_kl_from_ideal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_01388_amd.session import Session, mlp_init
    sess = Session(0)
    g = synth.chung_lu(n=2000, m=12000, seed=1)
    G = sess.graph(g.off, g.nbr)
    T = sess.tables(G, cv_seed=1, exact_cv=True)
    feats = sess.features(T)
    out = {}
    for name in ("triangle", "4-clique", "4-path", "diamond", "house", "4-cycle"):
        p = synth.named_pattern(name)
        c = compile_pattern(p.k, p.edges, mode="always")
        say(f"rooted counts {name}")
        ideal = judges.rooted_counts(g, p.k, p.edges, c["order"])
        row = {}
        q, tot = sess.step1_weights(G, T, p, mode="uniform")
        row["uniform"] = _kl(ideal, q, tot)
        for terms in ("f1", "f1_i1", "all"):
            q, tot = sess.step1_weights(G, T, p, mode="always", terms=terms)
            row[terms] = _kl(ideal, q, tot)
        # learned (a correction of f_approx trained on this graph's sampler output)
        steps = sess.weighted_steps(p, "learned")
        sums, counts = sess.learn_targets(G, T, p, 1 << 18, 3, mode="switch")
        base = sess.step_log_weights(T, p)
        rows = sess.learn_rows(sums, counts, step_mask=sum(1 << i for i in steps), min_count=2, base=base)
        tg = rows["target"].cpu().numpy()
        wt = rows["weight"].cpu().numpy()
        params = torch.from_numpy(mlp_init(5, float(np.average(tg, weights=wt)), zero_output=True)).to(sess.device)
        sess.mlp_train(params, feats, rows, epochs=200, batch=1024, lr=3e-3, seed=1)
        tabs = sess.learned_tables(params, feats, p, base=base)
        learned = {i: tab.data_ptr() for i, tab in tabs.items()}
        if 0 in tabs:
            q, tot = sess.step1_weights(G, T, p, mode="learned", learned=learned)
            row["learned"] = _kl(ideal, q, tot)
        out[name] = row
        say(f"KL {name}: " + ", ".join(f"{k} {v:.3g}" for k, v in row.items()))
    assert out["triangle"]["all"] < 1e-4
    for name, row in out.items():
        assert row["all"] < row["uniform"], name
    assert out["4-clique"]["f1_i1"] < 0.5 * out["4-clique"]["f1"]
    assert out["4-path"]["all"] < 0.5 * out["4-path"]["f1_i1"]
    T.close()
    G.close()
    sess.close()
