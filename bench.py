"""Benchmark of the AGIS sampling estimator on one MI355X.

Headline workload (the R-MAT scale 20 configuration): R-MAT scale 20
(2^20 vertices, edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised,
deduplicated, no self-loops; ~15.7M undirected edges) in symmetric CSR,
patterns 5-clique, 5-cycle, house and 4-star, f_approx with the paper's
switching rule (beta = 4/5), 10^8 samples per pattern.  The 10^8 samples of
each pattern are split into K consecutive index ranges; one step runs one
range of every pattern (one estimate each, its per-estimate tables
included, as the paper counts them in mining time), so the K steps together
are one 10^8-sample estimate per pattern.  ``value`` is samples per second
over the timed steps.

Also measured in the same run (the detail goes to a side file, a summary to
stderr): the roofline of the sampling kernel (request bytes counted per
sample by the metering kernel, against the HBM peak and against a measured
random-gather ceiling), time to +-1% relative error at 95% confidence
(Algorithm 1) per pattern for learned vs f_approx vs f_uniform, the batched
32-pattern runs, the term ablation and beta sweep, cliques on the degree
DAG, concentrations, the R-MAT scale 24 legs, and the CPU oracle timed on
the host's cores.  The last stdout line is one compact JSON object.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--detail PATH]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PATTERNS = ["5-clique", "5-cycle", "house", "4-star"]
C2_SAMPLES = 10 ** 8
HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_sample_rmat20_counters.json")
GOLDEN_5CLIQUE = os.path.join(ROOT, "tests", "golden", "rmat20_clique_counts.txt")
KERNEL_SOURCES = ["paper_2601_01388_amd/csrc/kernels.hip", "paper_2601_01388_amd/csrc/agis_common.h"]
GATHER_SIZES = [4, 16, 32, 64, 128, 256, 1024]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def rel_var(r) -> float:
    return r.variance / max(r.estimate ** 2, 1e-300)


def merge_results(rs):
    """(n, mean, population variance) of the union of several estimates'
    samples (Chan et al.'s pairwise update, in the given order)."""
    n, mean, m2 = 0.0, 0.0, 0.0
    for r in rs:
        nb, mb, m2b = float(r.n), r.estimate, r.variance * float(r.n)
        if nb == 0:
            continue
        if n == 0:
            n, mean, m2 = nb, mb, m2b
            continue
        tot = n + nb
        d = mb - mean
        mean += d * nb / tot
        m2 += m2b + d * d * n * nb / tot
        n = tot
    return n, mean, (m2 / n if n else 0.0)


def host_info() -> dict:
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model or platform.processor() or platform.machine(), "nproc": avail,
            "os_cpu_count": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def star_closed_form(g, leaves: int) -> int:
    """k-star embeddings: k! * sum_v C(d(v), k) (the paper's k-star example)."""
    d = np.diff(g.off).astype(np.int64)
    return int(sum(math.perm(int(x), leaves) for x in d[d >= leaves]))


def golden_cliques():
    """Exact clique counts of the R-MAT scale 20 bench graph (embeddings),
    written by tests/golden/make_rmat20_cliques.py from the oracle."""
    out = {}
    if os.path.exists(GOLDEN_5CLIQUE):
        for line in open(GOLDEN_5CLIQUE):
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[int(k)] = int(v)
    return out


def algorithmic_bytes(g, plan, recs) -> float:
    """Mean algorithmic HBM bytes per sample of the given records.

    Per sample: 16 B for the first draw (a prefix-table or offsets entry,
    +4 B for the weight of a weighted first step); for every later step that
    was reached, either the O(1) uniform single-backward draw -- 16 B of
    offsets, 4 B for the picked neighbour and 4*ceil(log2(d+1)) B per probe
    of an already matched vertex -- or, otherwise, the backward lists read
    in full (16 + 4 d(v_j) B each, merge model of the intersection) plus a
    16 B per-vertex record for every member of the intersection when the
    step draws from weights."""
    off = g.off
    deg = np.diff(off).astype(np.int64)
    k = plan.k
    total = 0.0
    for r in recs:
        steps = int(r["steps"])
        reached = steps + (1 if int(r["fail_step"]) >= 0 else 0)
        tau = [int(x) for x in r["v"][:steps]]
        b = 16.0 + (4.0 if plan.decision[0] and plan.f1[0] > 0 else 0.0)
        for i in range(1, min(reached, k)):
            bm = plan.bmask[i]
            weighted = plan.decision[i] and plan.f1[i] > 0
            js = [j for j in range(i) if bm >> j & 1]
            if not weighted and len(js) == 1:
                d = deg[tau[js[0]]]
                b += 20.0 + i * 4.0 * math.ceil(math.log2(d + 1))
            else:
                b += sum(16.0 + 4.0 * deg[tau[j]] for j in js)
                if weighted:
                    lists = [g.nbr[off[tau[j]]:off[tau[j] + 1]] for j in js]
                    inter = lists[0]
                    for other in lists[1:]:
                        inter = np.intersect1d(inter, other, assume_unique=True)
                    b += 16.0 * inter.size
        total += b
    return total / max(len(recs), 1)


def tune_batch(args, sess, G, T, pats, log):
    """Autotunes the launch for a batch leg on pilots of its own patterns (the
    launch shape that suits a batch of short to-eps rounds differs from the
    one for long single-pattern estimates); returns what was chosen."""
    if args.no_tune:
        return None
    tb = sess.autotune(G, T, pats, args.batch_tune_pilot, mode="switch")
    log(f"batch tuning: variant {tb.variant} grab {tb.grab} hub window {tb.hub_window}")
    return {"variant": tb.variant, "grab": tb.grab, "hub_window": tb.hub_window, "pilot_samples": args.batch_tune_pilot}


def is_star(p) -> bool:
    """A star: its steps after the centre are uniform draws from the centre's
    row under switching, which the library runs one sample per lane
    (k_sample_lanes)."""
    deg = [0] * p.k
    for a, b in p.edges:
        deg[a] += 1
        deg[b] += 1
    return p.k >= 2 and len(p.edges) == p.k - 1 and max(deg) == p.k - 1


def is_clique(p) -> bool:
    return len(p.edges) == p.k * (p.k - 1) // 2


class HostCSR:
    def __init__(self, off, nbr):
        self.off = off
        self.nbr = nbr


def cpu_baseline(g, c1, seconds_target: float):
    """The oracle on the host's cores (bounded samples of the bench's own
    workloads): the R-MAT scale 20 headline (the four patterns in switch
    mode on the symmetric graph, seed 7) single-threaded and with the OpenMP
    flavour on every core (one sampler per thread, contiguous index blocks),
    and the Chung-Lu C1 workload in full (triangle, 4-cycle, 4-clique x
    uniform, switch, always, 10^6 samples each) on every core."""
    import oracle
    from oracle.pattern import compile_pattern
    import synth
    info = host_info()
    threads = int(info["omp_num_threads"] or 0) or info["nproc"]
    log(f"cpu baseline: oracle tables of R-MAT-20 on {threads} threads (setup, untimed)")
    t = oracle.Tables(g, cv_seed=1, threads=threads)
    samplers = [oracle.Sampler(g, t, compile_pattern(p.k, p.edges, mode="switch"), seed=7, pattern_id=pid)
                for pid, p in enumerate(synth.named_pattern(n) for n in PATTERNS)]
    per = []
    for s in samplers:
        t0 = time.perf_counter()
        s.run(0, 100)
        per.append((time.perf_counter() - t0) / 100)
    n1 = max(100, int(0.35 * seconds_target / max(sum(per), 1e-9)))
    t0 = time.perf_counter()
    for s in samplers:
        s.run(0, n1)
    el1 = time.perf_counter() - t0
    nall = max(n1, int(0.35 * seconds_target * threads / max(sum(per), 1e-9)))
    t0 = time.perf_counter()
    used = threads
    means = {}
    for name, s in zip(PATTERNS, samplers):
        st, used = s.run_parallel(0, nall, threads=threads)
        means[name] = st.mean
    elall = time.perf_counter() - t0
    # C1 in full on every core
    tc = oracle.Tables(c1, cv_seed=1, threads=threads)
    c1_runs = {}
    t0 = time.perf_counter()
    for pid, name in enumerate(("triangle", "4-cycle", "4-clique")):
        p = synth.named_pattern(name)
        for mode in ("uniform", "switch", "always"):
            st, _ = oracle.Sampler(c1, tc, compile_pattern(p.k, p.edges, mode=mode), seed=7,
                                   pattern_id=pid).run_parallel(0, 10 ** 6, threads=threads)
            c1_runs[f"{name}/{mode}"] = {"mean": st.mean, "n": int(st.n)}
    elc1 = time.perf_counter() - t0
    return {
        "value": len(PATTERNS) * nall / elall,
        "unit": "samples/s",
        "cores": used,
        "kind": "oracle",
        "sample": (f"R-MAT-20 headline workload (5-clique, 5-cycle, house, 4-star; switch; seed 7): first {nall} "
                   f"sample indices per pattern with the OpenMP oracle on {used} threads ({elall:.1f} s); "
                   f"single-threaded: first {n1} per pattern ({el1:.1f} s)"),
        "single_thread_value": len(PATTERNS) * n1 / el1,
        "rmat20_samples_per_pattern": nall,
        "rmat20_means": means,
        "c1_full": {"samples": 9 * 10 ** 6, "seconds": elc1, "threads": used, "samples_per_s": 9e6 / elc1,
                    "runs": c1_runs},
        "host": info,
    }


GATHER_BUFFERS = {"128MiB": 1 << 27, "8GiB": 1 << 33}


def gather_ceiling(sess, waves_per_cu: int):
    """Random-gather ceiling (agis_gather_bench) for segment sizes of 4 B to
    1 KiB, as chains of dependent reads and as independent reads, at the
    sampler's resident waves per compute unit, over two footprints: 128 MiB
    (held by the 256 MB Infinity Cache) and 8 GiB (HBM)."""
    import torch
    out = {}
    for label, nbytes in GATHER_BUFFERS.items():
        buf = torch.arange(nbytes // 8, dtype=torch.int64, device=sess.device)
        rows = {}
        for S in GATHER_SIZES:
            row = {}
            for dep in (True, False):
                sec, ub = sess.gather_bench(buf, S, dep, waves_per_cu=waves_per_cu, rounds=32, seed=S)
                rounds = int(min(max(32 * 0.02 / max(sec, 1e-6), 32), 200000))
                sec, ub = sess.gather_bench(buf, S, dep, waves_per_cu=waves_per_cu, rounds=rounds, seed=S + 1)
                row["dependent_gbs" if dep else "independent_gbs"] = ub / sec / 1e9
            rows[S] = row
        out[label] = rows
        del buf
        torch.cuda.empty_cache()
    return out


def learned_four(args, sess, T, pats):
    """One MLP per headline pattern, trained on extension counts the sampler
    produces on R-MAT scale 18 (seed 18), BF16 inference into pick tables
    for the bench graph (residual: a learned correction of f_approx)."""
    import torch
    import synth
    from paper_2601_01388_amd.session import mlp_init
    learned = {}
    log("learned proposal: training graph R-MAT scale 18")
    gtr = synth.rmat(18, 16, seed=18)
    Gtr = sess.graph(gtr.off, gtr.nbr)
    Ttr = sess.tables(Gtr, cv_seed=1)
    ftr = sess.features(Ttr)
    fev = sess.features(T)
    residual = not args.learned_absolute
    batch_rows = 4096
    for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
        t0 = time.perf_counter()
        steps = sess.weighted_steps(p, "learned")
        sums, counts = sess.learn_targets(Gtr, Ttr, p, args.train_samples, 101 + pid, mode="switch")
        base_tr = sess.step_log_weights(Ttr, p) if residual else None
        rows = sess.learn_rows(sums, counts, step_mask=sum(1 << i for i in steps), min_count=2, base=base_tr)
        del sums, counts, base_tr
        tg = rows["target"].cpu().numpy()
        wt = rows["weight"].cpu().numpy()
        init = mlp_init(7 + pid, float(np.average(tg, weights=wt)) if rows["rows"] else 0.0, zero_output=residual)
        params = torch.from_numpy(init).to(sess.device)
        per_epoch = max(1, -(-rows["rows"] // batch_rows))
        epochs = max(args.train_epochs, -(-args.train_min_steps // per_epoch))
        losses = sess.mlp_train(params, ftr, rows, epochs=epochs, batch=batch_rows, lr=3e-3, seed=pid)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        base_ev = sess.step_log_weights(T, p) if residual else None
        tabs = sess.learned_tables(params, fev, p, base=base_ev, rows=rows)
        del base_ev
        torch.cuda.synchronize()
        infer_s = time.perf_counter() - t0
        learned[name] = {"tables": tabs, "ptrs": {i: tab.data_ptr() for i, tab in tabs.items()},
                         "info": {"train_rows": rows["rows"], "train_seconds": train_s, "epochs": epochs,
                                  "adam_steps": epochs * per_epoch, "residual": residual,
                                  "loss_first_last": [losses[0], losses[-1]] if losses else None,
                                  "infer_seconds": infer_s, "weighted_steps": steps}}
        log(f"learned {name}: {rows['rows']} rows, {epochs} epochs, train {train_s:.2f} s, loss "
            f"{losses[0]:.3g} -> {losses[-1]:.3g}, tables {infer_s * 1e3:.1f} ms")
    Ttr.close()
    Gtr.close()
    return learned


def time_to_eps(args, sess, G, T, pats, learned):
    """Time to +-1% at 95% CI (Algorithm 1) per pattern and proposal; checks
    every 4096 samples from 4096 on, so that the stop point reflects the
    proposal rather than the check interval; budget --eps-budget.  (These
    one-launch runs keep the 5-clique's launch shape: the per-pattern shapes
    are tuned on fixed-size launches, and the run-to-eps kernel at 7 waves
    per SIMD reached +-1% later on the 5-cycle and the house.)"""
    table = {}
    ck = args.eps_check
    for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
        for mode in ("learned", "switch", "always", "uniform"):
            if mode == "learned" and name not in learned:
                continue
            kw = dict(learned=learned[name]["ptrs"]) if mode == "learned" else {}
            r = sess.estimate(G, T, p, args.eps_budget, 11, mode=mode, pattern_id=pid, eps=0.01, delta=0.05,
                              check_every=ck, min_samples=ck, **kw)
            need = r.n * (r.eps_hat / 0.01) ** 2 if math.isfinite(r.eps_hat) else None
            label = {"switch": "f_approx", "always": "f_approx_always", "uniform": "f_uniform",
                     "learned": "learned"}[mode]
            entry = {"seconds": r.seconds, "converged": bool(r.converged), "samples": r.n, "estimate": r.estimate,
                     "eps_hat": r.eps_hat, "rel_var": rel_var(r), "samples_needed": need,
                     "stopped_at_first_check": r.n <= ck}
            if mode == "learned":
                entry["seconds_incl_table_inference"] = r.seconds + learned[name]["info"]["infer_seconds"]
                entry.update({k: v for k, v in learned[name]["info"].items() if k != "weighted_steps"})
            table[f"{name}/{label}"] = entry
            log(f"+-1% {name} {label}: {r.seconds:.4f} s, n={r.n}, rel.var {entry['rel_var']:.4g}, "
                f"converged={bool(r.converged)}")
    for pid, name in enumerate(PATTERNS):
        if f"{name}/learned" not in table:
            continue
        table[f"{name}/learned"]["rel_var_vs_f_approx"] = (
            table[f"{name}/learned"]["rel_var"] / max(table[f"{name}/f_approx"]["rel_var"], 1e-300))
        t0 = time.perf_counter()
        pl = sess.estimate(G, T, pats[pid], args.pilot_samples, 97, mode="learned", pattern_id=pid,
                           learned=learned[name]["ptrs"])
        pa = sess.estimate(G, T, pats[pid], args.pilot_samples, 97, mode="switch", pattern_id=pid)
        pilot_s = time.perf_counter() - t0
        keep = rel_var(pl) < rel_var(pa)
        chosen = table[f"{name}/learned" if keep else f"{name}/f_approx"]
        table[f"{name}/learned_with_fallback"] = {
            "chosen": "learned" if keep else "f_approx", "pilot_seconds": pilot_s,
            "seconds": chosen["seconds"] + pilot_s, "samples": chosen["samples"],
            "converged": chosen["converged"], "estimate": chosen["estimate"], "rel_var": chosen["rel_var"]}
        log(f"{name}: pilot keeps {'learned' if keep else 'f_approx'}")
    return table


def ablation_leg(args, sess, G, T):
    """Incremental terms of f_approx and the switching threshold beta (the
    paper's analysis of the approximation and of beta)."""
    import synth
    z2 = 1.959963984540054 ** 2
    ab = {"samples": args.ablation_samples, "terms": {}, "beta": {}}
    t0 = time.perf_counter()
    for name in ["4-clique", "4-path", "5-clique", "5-cycle", "house"]:
        p = synth.named_pattern(name)
        row = {}
        for terms in ("f1", "f1_i1", "all"):
            r = sess.estimate(G, T, p, args.ablation_samples, 17, mode="switch", terms=terms)
            rv = rel_var(r)
            row[terms] = {"rel_var": rv, "samples_needed": z2 * rv / 1e-4, "estimate": r.estimate,
                          "seconds_per_sample": r.seconds / r.n}
        ab["terms"][name] = row
    betas = [("-inf", (-1, 0)), ("1/2", (1, 2)), ("4/5", (4, 5)), ("5/6", (5, 6)), ("1", (1, 1)), ("+inf", (1, 0))]
    for name in ["house", "5-cycle", "6-cycle", "chordal-7-cycle"]:
        p = synth.named_pattern(name)
        row = {}
        for label, beta in betas:
            r = sess.estimate(G, T, p, args.ablation_samples, 19, mode="switch", beta=beta)
            rv = rel_var(r)
            row[label] = {"rel_var": rv, "samples_needed": z2 * rv / 1e-4, "estimate": r.estimate,
                          "seconds_per_sample": r.seconds / r.n,
                          "uniform_steps": int(sum(1 for i in range(p.k) if not r.plan.decision[i]))}
        ab["beta"][name] = row
    ab["seconds"] = time.perf_counter() - t0
    log(f"term ablation and beta sweep: {ab['seconds']:.1f} s")
    for name, row in ab["terms"].items():
        log("  terms " + name + ": " + ", ".join(f"{k} {v['rel_var']:.3g}" for k, v in row.items()))
    for name, row in ab["beta"].items():
        log("  beta " + name + ": " + ", ".join(f"{k} {v['rel_var']:.3g}" for k, v in row.items()))
    return ab


def batch_leg(args, sess, G, T, restore_tuning):
    """32 connected patterns of 4-7 vertices (seed 3) with budgets
    log-uniform in [10^6, 10^9], all run to +-1% in one batched run, and
    the same 32 runs one estimate at a time for comparison."""
    import torch
    import synth
    pset = synth.random_pattern_set(32, seed=3)
    bpats = [p for p, _ in pset]
    budgets = [max(1, int(b * args.batch_budget_scale)) for _, b in pset]
    log(f"32-pattern batch to +-1%, total budget {sum(budgets):.3g} samples")
    btune = tune_batch(args, sess, G, T, bpats, log)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sess.estimate_batch(G, T, bpats, budgets, 13, mode="switch", eps=0.01, delta=0.05,
                              check_every=1 << 16, min_samples=1 << 14)
    torch.cuda.synchronize()
    bt = time.perf_counter() - t0
    # the same 32 runs one estimate at a time (what the batch replaces)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    one = [sess.estimate(G, T, p, b, 13, mode="switch", eps=0.01, delta=0.05, check_every=1 << 16,
                         min_samples=1 << 14, pattern_id=pid) for pid, (p, b) in enumerate(zip(bpats, budgets))]
    torch.cuda.synchronize()
    st = time.perf_counter() - t0
    restore_tuning()
    log(f"the same 32 runs one at a time: {st:.2f} s, {sum(r.n for r in one):.3g} samples")
    out = {"patterns": 32, "tuning": btune, "seconds": bt, "one_at_a_time_seconds": st,
           "one_at_a_time_samples": int(sum(r.n for r in one)), "samples": int(sum(r.n for r in res)),
           "converged": int(sum(r.converged for r in res)), "samples_per_s": sum(r.n for r in res) / bt,
           "budget_total": int(sum(budgets)),
           "per_pattern": [{"k": p.k, "edges": len(p.edges), "budget": b, "samples": r.n,
                            "converged": bool(r.converged), "seconds": r.seconds, "rel_var": rel_var(r)}
                           for p, b, r in zip(bpats, budgets, res)]}
    log(f"batch: {bt:.2f} s, {out['converged']}/32 converged, {out['samples']:.3g} samples")
    return out


def oriented_leg(args, sess, G, T):
    """4- and 5-cliques on the degree-oriented graph vs the symmetric graph."""
    import torch
    import synth
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    O = sess.orient(G)
    TO = sess.tables(O, cv_seed=1)
    torch.cuda.synchronize()
    out = {"orient_and_tables_ms": 1e3 * (time.perf_counter() - t0), "nnz": O.nnz, "patterns": {}}
    for k in (4, 5):
        p = synth.patterns.clique(k)
        row = {}
        for label, (gg, tt) in (("oriented", (O, TO)), ("symmetric", (G, T))):
            r = sess.estimate(gg, tt, p, args.samples_oriented, 29, mode="switch", pattern_id=k)
            e = sess.estimate(gg, tt, p, args.eps_budget, 31, mode="switch", pattern_id=k, eps=0.01, delta=0.05,
                              check_every=args.eps_check, min_samples=args.eps_check)
            row[label] = {"samples_per_s_kernel": r.n / max(r.sample_kernel_seconds, 1e-12), "rel_var": rel_var(r),
                          "estimate": r.estimate, "time_to_1pct_s": e.seconds, "samples_to_1pct": e.n,
                          "converged": bool(e.converged)}
        out["patterns"][f"{k}-clique"] = row
        log(f"{k}-clique oriented: {row['oriented']['samples_per_s_kernel']:.3g} samples/s, rel.var "
            f"{row['oriented']['rel_var']:.3g}, +-1% in {row['oriented']['time_to_1pct_s']:.4f} s; symmetric: "
            f"{row['symmetric']['samples_per_s_kernel']:.3g} samples/s, rel.var {row['symmetric']['rel_var']:.3g}, "
            f"+-1% in {row['symmetric']['time_to_1pct_s']:.4f} s")
    TO.close()
    O.close()
    return out


def conc_leg(args, sess, G, T):
    """Concentrations of all connected 4- and 5-vertex patterns, each run to
    +-1% inside batched runs (the paper's comparison with MCMC)."""
    import torch
    out = {}
    for k in (4, 5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = sess.concentrations(G, T, k, args.conc_budget, 23, mode="switch", eps=0.01, delta=0.05,
                                check_every=1 << 16, min_samples=1 << 14)
        torch.cuda.synchronize()
        ct = time.perf_counter() - t0
        res = c["results"]
        out[f"k{k}"] = {
            "patterns": len(res), "seconds": ct, "budget_per_pattern": args.conc_budget,
            "converged": int(sum(r.converged for r in res)), "samples": int(sum(r.n for r in res)),
            "per_pattern": [{"edges": [list(e) for e in p[1]], "copies": r.copies, "eps_hat": r.eps_hat,
                             "conc_edge": float(ce), "conc_induced": float(ci), "induced": float(ind)}
                            for p, r, ce, ci, ind in zip(c["patterns"], res, c["conc_edge"], c["conc_induced"],
                                                          c["induced"])]}
        log(f"concentrations k={k}: {len(res)} patterns, {out[f'k{k}']['converged']} converged, {ct:.2f} s")
    return out


def c1_gpu_leg(sess, c1):
    """The Chung-Lu C1 workload on the GPU: triangle, 4-cycle, 4-clique under
    uniform, switch and always, 10^6 samples each, seed 7."""
    import synth
    G = sess.graph(c1.off, c1.nbr)
    T = sess.tables(G, cv_seed=1)
    out = {}
    t_all = 0.0
    for pid, name in enumerate(("triangle", "4-cycle", "4-clique")):
        p = synth.named_pattern(name)
        for mode in ("uniform", "switch", "always"):
            r = sess.estimate(G, T, p, 10 ** 6, 7, mode=mode, pattern_id=pid)
            out[f"{name}/{mode}"] = {"estimate": r.estimate, "rel_var": rel_var(r), "seconds": r.seconds}
            t_all += r.seconds
    T.close()
    G.close()
    return {"runs": out, "seconds": t_all, "samples_per_s": 9e6 / t_all}


def bpats_budgets(args):
    import synth
    pset = synth.random_pattern_set(32, seed=3)
    return [p for p, _ in pset], [max(1, int(b * args.large_budget_scale)) for _, b in pset]


def large_legs(args, sess, G20, T20, pats_budgets, log, restore_tuning):
    import torch
    import synth
    from paper_2601_01388_amd.session import mlp_init
    bpats, budgets = pats_budgets
    out = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off, nbr = synth.graphs.rmat_device(24, 16, seed=24, device=str(sess.device))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    G = sess.graph(off, nbr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = sess.tables(G, cv_seed=1)
    torch.cuda.synchronize()
    tables_s = time.perf_counter() - t0
    dmax = int((off[1:] - off[:-1]).max().item())
    out["graph"] = {"scale": 24, "seed": 24, "generator": "torch GPU Philox stream", "n": G.n, "nnz": G.nnz,
                    "dmax": dmax, "generate_s": gen_s, "tables_ms": 1e3 * tables_s}
    log(f"R-MAT scale 24: n={G.n} nnz={G.nnz} dmax={dmax}; generated in {gen_s:.1f} s, tables {1e3 * tables_s:.1f} ms")
    log(f"32-pattern batch on scale 24 to +-1%, total budget {sum(budgets):.3g} samples")
    btune = tune_batch(args, sess, G, T, bpats, log)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = sess.estimate_batch(G, T, bpats, budgets, 13, mode="switch", eps=0.01, delta=0.05,
                              check_every=1 << 16, min_samples=1 << 14)
    torch.cuda.synchronize()
    bt = time.perf_counter() - t0
    restore_tuning()
    out["batch_32_patterns"] = {
        "tuning": btune, "budget_scale": args.large_budget_scale, "seconds": bt, "samples": int(sum(r.n for r in res)), "converged": int(sum(r.converged for r in res)),
        "samples_per_s": sum(r.n for r in res) / bt, "budget_total": int(sum(budgets)),
        "per_pattern": [{"k": p.k, "edges": len(p.edges), "budget": b, "samples": r.n,
                         "converged": bool(r.converged), "seconds": r.seconds,
                         "rel_var": r.variance / max(r.estimate ** 2, 1e-300)}
                        for p, b, r in zip(bpats, budgets, res)]}
    log(f"scale-24 batch: {bt:.2f} s, {out['batch_32_patterns']['converged']}/32 converged, "
        f"{out['batch_32_patterns']['samples']:.3g} samples")
    # learned proposal per pattern: trained on scale-20 targets, evaluated here
    f20 = sess.features(T20)
    f24 = sess.features(T)
    rows_out = []
    ratios = []
    fb_ratios = []
    t0 = time.perf_counter()
    for pid, p in enumerate(bpats):
        steps = sess.weighted_steps(p, "learned")
        if not steps:
            rows_out.append({"k": p.k, "edges": len(p.edges), "weighted_steps": 0})
            continue
        sums, counts = sess.learn_targets(G20, T20, p, 1 << 19, 301 + pid, mode="switch")
        rows = sess.learn_rows(sums, counts, step_mask=sum(1 << i for i in steps), min_count=2,
                               base=sess.step_log_weights(T20, p))
        del sums, counts
        if rows["rows"] == 0:
            rows_out.append({"k": p.k, "edges": len(p.edges), "weighted_steps": len(steps), "train_rows": 0})
            continue
        tg = rows["target"].cpu().numpy()
        wt = rows["weight"].cpu().numpy()
        params = torch.from_numpy(mlp_init(11 + pid, float(np.average(tg, weights=wt)), zero_output=True)).to(
            sess.device)
        per_epoch = max(1, -(-rows["rows"] // 4096))
        sess.mlp_train(params, f20, rows, epochs=max(20, -(-1500 // per_epoch)), batch=4096, lr=3e-3, seed=pid)
        tabs = sess.learned_tables(params, f24, p, base=sess.step_log_weights(T, p), rows=rows)
        ptrs = {i: tab.data_ptr() for i, tab in tabs.items()}
        rl = sess.estimate(G, T, p, args.large_eval_samples, 41, mode="learned", learned=ptrs, pattern_id=pid)
        ra = sess.estimate(G, T, p, args.large_eval_samples, 41, mode="switch", pattern_id=pid)
        vl = rl.variance / max(rl.estimate ** 2, 1e-300)
        va = ra.variance / max(ra.estimate ** 2, 1e-300)
        # fallback: pilots of each mode on other samples keep the learned
        # tables only where their variance per sample is lower
        pl = sess.estimate(G, T, p, args.pilot_samples, 43, mode="learned", learned=ptrs, pattern_id=pid)
        pa = sess.estimate(G, T, p, args.pilot_samples, 43, mode="switch", pattern_id=pid)
        keep = pl.variance / max(pl.estimate ** 2, 1e-300) < pa.variance / max(pa.estimate ** 2, 1e-300)
        entry = {"k": p.k, "edges": len(p.edges), "weighted_steps": len(steps), "train_rows": rows["rows"],
                 "rel_var_learned": vl, "rel_var_f_approx": va, "estimate_learned": rl.estimate,
                 "estimate_f_approx": ra.estimate, "pilot_keeps_learned": bool(keep)}
        if va > 0 and vl > 0:
            entry["learned_over_f_approx"] = vl / va
            ratios.append(vl / va)
            fb_ratios.append(vl / va if keep else 1.0)
        rows_out.append(entry)
        del tabs, params, rows
    learned_s = time.perf_counter() - t0
    geo = float(np.exp(np.mean(np.log(ratios)))) if ratios else None
    geo_fb = float(np.exp(np.mean(np.log(fb_ratios)))) if fb_ratios else None
    out["learned_32_patterns"] = {"train_graph": "R-MAT scale 20 (the bench graph)", "eval_samples": args.large_eval_samples,
                                  "pilot_samples": args.pilot_samples, "seconds": learned_s,
                                  "geomean_rel_var_learned_over_f_approx": geo,
                                  "geomean_rel_var_with_fallback_over_f_approx": geo_fb,
                                  "patterns_better": int(sum(r < 1 for r in ratios)), "patterns_compared": len(ratios),
                                  "per_pattern": rows_out}
    log(f"learned on scale 24: geomean variance ratio learned/f_approx {geo} ({geo_fb} with the pilot fallback), "
        f"{out['learned_32_patterns']['patterns_better']}/{len(ratios)} better, {learned_s:.1f} s")
    T.close()
    G.close()
    del off, nbr
    torch.cuda.empty_cache()
    return out


def c5_leg(args, sess):
    """R-MAT scale 30 (2^30 vertices, edge factor 16, ~3.4e10 CSR slots)
    resident in HBM, generated on the GPU (synth.graphs.rmat_gpu, seed 30):
    5-clique, 6-cycle and the chordal 7-cycle run to +-1% at 95% CI under
    learned, f_approx (switching and always) and f_uniform, each run capped
    at --c5-seconds of wall time (the cancel flag stops it between rounds
    and the partial result reports the error it reached), then the 32-pattern
    batch to +-1% in one launch under --c5-batch-seconds; the 4-star and
    3-path closed forms and cross-mode agreement are the judges."""
    import ctypes
    import threading
    import torch
    import synth
    from synth import graphs
    from paper_2601_01388_amd.session import mlp_init
    out = {}

    def mem():
        free, total = torch.cuda.mem_get_info()
        return round(free / 2 ** 30, 1)

    t0 = time.perf_counter()
    off, nbr = graphs.rmat_gpu(30, 16, seed=30, device=str(sess.device))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    G = sess.graph(off, nbr, validate=True)
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    T = sess.tables(G, cv_seed=1)
    torch.cuda.synchronize()
    tables_s = time.perf_counter() - t0
    d = (off[1:] - off[:-1]).double()
    dmax = int(d.max().item())
    out["graph"] = {"scale": 30, "seed": 30, "generator": "counter-based R-MAT on the GPU (synth.graphs.rmat_gpu)",
                    "n": G.n, "nnz": G.nnz, "dmax": dmax, "generate_s": gen_s, "load_validate_s": load_s,
                    "tables_s": tables_s, "neighbour_bytes": 4 * G.nnz, "offset_bytes": 8 * (G.n + 1),
                    "free_gib_after_tables": mem()}
    log(f"C5: R-MAT scale 30 n={G.n} nnz={G.nnz} dmax={dmax}; generated {gen_s:.1f} s, loaded+validated "
        f"{load_s:.1f} s, tables {tables_s:.1f} s, free {mem()} GiB")
    sentinels = {}
    exact4 = float((d * (d - 1) * (d - 2) * (d - 3)).sum().item())
    exact3p = float((d * (d - 1)).sum().item())  # wedges: 2! x sum C(d, 2)
    for name, exact in (("4-star", exact4), ("wedge", exact3p)):
        p = synth.named_pattern(name)
        r = sess.estimate(G, T, p, 1 << 22, 5, mode="switch")
        se = math.sqrt(r.variance / r.n)
        sentinels[name] = {"estimate": r.estimate, "exact": exact, "z": (r.estimate - exact) / se if se else 0.0,
                           "rel_err": (r.estimate - exact) / exact}
        log(f"C5 {name}: {r.estimate:.6g} vs closed form {exact:.6g} (z {sentinels[name]['z']:.2f})")
    out["sentinels"] = sentinels
    # the degree arithmetic's temporaries (8 GiB each) go back to the device:
    # the sampler's scratch budget is a share of the free memory
    del d
    torch.cuda.empty_cache()
    # learned tables: one network per pattern trained on extension counts of
    # the R-MAT scale 20 graph, inferred on this graph's features.  The
    # non-learned modes run first, with nothing else resident: a wave's
    # scratch holds a maximum-degree list here (48 MB), so the free memory
    # sets the number of waves, and the features (16 GiB) and a pattern's
    # learned tables (4 GiB per weighted step) are built only for its
    # learned run and freed after it.
    g20 = synth.rmat(20, 16, seed=20)
    G20 = sess.graph(g20.off, g20.nbr)
    T20 = sess.tables(G20, cv_seed=1)
    f20 = sess.features(T20)
    names = ("5-clique", "6-cycle", "chordal-7-cycle")
    labels = {"switch": "f_approx", "always": "f_approx_always", "uniform": "f_uniform", "learned": "learned"}
    runs = {name: {} for name in names}

    def run_mode(pid, name, p, mode, kw):
        free_before = mem()
        flag = ctypes.c_int32(0)
        timer = threading.Timer(args.c5_seconds, lambda f=flag: setattr(f, "value", 1))
        timer.start()
        r = sess.estimate(G, T, p, args.c5_budget, 61 + pid, mode=mode, pattern_id=pid, eps=0.01, delta=0.05,
                          check_every=1 << 14, min_samples=1 << 14, cancel=flag, **kw)
        timer.cancel()
        label = labels[mode]
        need = r.n * (r.eps_hat / 0.01) ** 2 if r.n and math.isfinite(r.eps_hat) else None
        runs[name][label] = {"seconds": r.seconds, "samples": r.n, "converged": bool(r.converged),
                             "stopped_by_time_cap": r.status == -9, "estimate": r.estimate, "eps_hat": r.eps_hat,
                             "rel_var": rel_var(r) if r.n else None, "samples_needed": need,
                             "samples_per_s": r.n / r.seconds if r.seconds > 0 else None,
                             "free_gib_before": free_before}
        log(f"C5 +-1% {name} {label}: {r.seconds:.1f} s, n={r.n}, eps_hat {r.eps_hat:.4f}, "
            f"converged={bool(r.converged)}, estimate {r.estimate:.6g} ({free_before} GiB free before)")

    for pid, name in enumerate(names):
        p = synth.named_pattern(name)
        for mode in ("switch", "always", "uniform"):
            run_mode(pid, name, p, mode, {})
    # the sampler's kept scratch (sized to half of the free memory) goes
    # back before the features and learned tables are allocated
    sess.release_scratch()
    for pid, name in enumerate(names):
        p = synth.named_pattern(name)
        steps = sess.weighted_steps(p, "learned")
        sums, counts = sess.learn_targets(G20, T20, p, 1 << 20, 501 + pid, mode="switch")
        rows = sess.learn_rows(sums, counts, step_mask=sum(1 << i for i in steps), min_count=2,
                               base=sess.step_log_weights(T20, p))
        del sums, counts
        tg = rows["target"].cpu().numpy()
        wt = rows["weight"].cpu().numpy()
        params = torch.from_numpy(mlp_init(31 + pid, float(np.average(tg, weights=wt)) if rows["rows"] else 0.0,
                                           zero_output=True)).to(sess.device)
        per_epoch = max(1, -(-rows["rows"] // 4096))
        sess.mlp_train(params, f20, rows, epochs=max(20, -(-1500 // per_epoch)), batch=4096, lr=3e-3, seed=pid)
        f30 = sess.features(T)
        base = sess.step_log_weights(T, p)
        tabs = sess.learned_tables(params, f30, p, base=base, rows=rows)
        del base, f30
        torch.cuda.empty_cache()
        ptrs = {i: tab.data_ptr() for i, tab in tabs.items()}
        run_mode(pid, name, p, "learned", dict(learned=ptrs))
        sess.release_scratch()
        del tabs, params, rows
        torch.cuda.empty_cache()
    for name in names:
        row = runs[name]
        # cross-mode agreement of the estimates (each with its own standard error)
        labs = [k for k in row if row[k]["samples"]]
        worst = 0.0
        for a in labs:
            for b in labs:
                if a < b:
                    ra, rb = row[a], row[b]
                    se = math.sqrt(ra["rel_var"] * ra["estimate"] ** 2 / ra["samples"]
                                   + rb["rel_var"] * rb["estimate"] ** 2 / rb["samples"])
                    if se > 0:
                        worst = max(worst, abs(ra["estimate"] - rb["estimate"]) / se)
        row["max_cross_mode_z"] = worst
    out["to_1pct"] = runs
    # the 32-pattern batch (seed 3, budgets log-uniform in [10^6, 10^9]) to
    # +-1% in one launch, capped at --c5-batch-seconds through the cancel flag
    pset = synth.random_pattern_set(32, seed=3)
    bp, bb = [q for q, _ in pset], [b for _, b in pset]
    flag = ctypes.c_int32(0)
    timer = threading.Timer(args.c5_batch_seconds, lambda f=flag: setattr(f, "value", 1))
    t0 = time.perf_counter()
    timer.start()
    res = sess.estimate_batch(G, T, bp, bb, 13, mode="switch", eps=0.01, delta=0.05, check_every=1 << 14,
                              min_samples=1 << 14, cancel=flag)
    timer.cancel()
    bt = time.perf_counter() - t0
    out["batch_32_patterns"] = {
        "seconds": bt, "cap_seconds": args.c5_batch_seconds, "stopped_by_time_cap": res[0].status == -9,
        "samples": int(sum(r.n for r in res)), "converged": int(sum(r.converged for r in res)),
        "per_pattern": [{"k": q.k, "edges": len(q.edges), "budget": b, "samples": r.n, "converged": bool(r.converged),
                         "seconds": r.seconds, "eps_hat": r.eps_hat} for q, b, r in zip(bp, bb, res)]}
    log(f"C5 32-pattern batch: {bt:.1f} s, {out['batch_32_patterns']['converged']}/32 converged, "
        f"{out['batch_32_patterns']['samples']:.3g} samples")
    out["free_gib_end"] = mem()
    T20.close()
    G20.close()
    T.close()
    G.close()
    del off, nbr, f20
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--total-samples", type=int, default=C2_SAMPLES,
                    help="samples per pattern over all timed steps (the R-MAT scale 20 configuration: 10^8)")
    ap.add_argument("--detail", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="side file for the full per-leg detail")
    ap.add_argument("--eps-budget", type=int, default=10 ** 8, help="sample budget of each run to +-1%%")
    ap.add_argument("--eps-check", type=int, default=4096, help="check interval (and minimum) of the +-1%% runs")
    ap.add_argument("--headline-only", action="store_true", help="only the timed steps and their roofline")
    ap.add_argument("--skip-eps", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="wall seconds of the R-MAT-20 oracle samples")
    ap.add_argument("--meter-samples", type=int, default=4096, help="samples metered per pattern for the roofline")
    ap.add_argument("--bytes-records", type=int, default=1000, help="records per pattern priced by the merge model")
    ap.add_argument("--skip-gather", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run 3 plain device copies of this many bytes (counter calibration) and exit")
    ap.add_argument("--tune-pilot", type=int, default=1 << 20, help="pilot samples per pattern of the autotuner")
    ap.add_argument("--batch-tune-pilot", type=int, default=1 << 15,
                    help="pilot samples per pattern of the batch legs' autotuning")
    ap.add_argument("--samples-oriented", type=int, default=1 << 22)
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
    ap.add_argument("--skip-ablation", action="store_true")
    ap.add_argument("--skip-conc", action="store_true")
    ap.add_argument("--skip-oriented", action="store_true")
    ap.add_argument("--skip-c1", action="store_true")
    ap.add_argument("--c5", action="store_true",
                    help="only the R-MAT scale 30 leg (3.4e10 CSR slots resident in HBM); prints its own JSON line")
    ap.add_argument("--c5-seconds", type=float, default=40.0, help="wall-time cap of each C5 run to +-1%%")
    ap.add_argument("--c5-budget", type=int, default=1 << 31, help="sample budget of each C5 run to +-1%%")
    ap.add_argument("--c5-batch-seconds", type=float, default=60.0,
                    help="wall-time cap of the C5 32-pattern batch to +-1%%")
    ap.add_argument("--conc-budget", type=int, default=20_000_000,
                    help="sample budget per pattern of the concentration runs (to +-1%%)")
    ap.add_argument("--skip-large", action="store_true",
                    help="skip the R-MAT scale 24 legs (32-pattern batch; learned proposal trained on scale 20)")
    ap.add_argument("--large-budget-scale", type=float, default=1.0,
                    help="multiplier on the 32-pattern budgets on R-MAT scale 24 (1.0 = the full budgets)")
    ap.add_argument("--large-eval-samples", type=int, default=1 << 20,
                    help="samples per pattern and mode for the learned-vs-f_approx variance on scale 24")
    ap.add_argument("--ablation-samples", type=int, default=1 << 20,
                    help="samples per configuration of the term-ablation and beta sweeps")
    ap.add_argument("--train-samples", type=int, default=1 << 20, help="sampler runs producing training targets")
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--train-min-steps", type=int, default=1500, help="fewest Adam steps per pattern")
    ap.add_argument("--learned-absolute", action="store_true",
                    help="learned tables predict the log weight itself instead of correcting f_approx")
    ap.add_argument("--pilot-samples", type=int, default=1 << 18,
                    help="per-mode pilot deciding between learned and f_approx")
    ap.add_argument("--batch-budget-scale", type=float, default=1.0,
                    help="multiplier on the 32-pattern set's budgets (log-uniform in [1e6, 1e9])")
    args = ap.parse_args()
    if args.headline_only:
        args.skip_eps = args.skip_cpu = args.skip_batch = args.skip_learned = args.skip_ablation = True
        args.skip_conc = args.skip_oriented = args.skip_large = args.skip_c1 = True

    if args.copy_calibration:
        # a plain device copy of known size, for scaling hardware byte counters
        import torch
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": n * 4, "copies": 3}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(samples are independent: more GPUs would split the sample index range)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2601_01388_amd.session import Session

    if args.c5:
        sess = Session(0)
        c5 = c5_leg(args, sess)
        sess.close()
        try:
            os.makedirs(os.path.dirname(args.detail), exist_ok=True)
            with open(args.detail, "w") as f:
                json.dump({"c5": c5}, f, indent=1, default=float)
        except OSError as e:
            log(f"could not write the detail file: {e}")
        print(json.dumps({"c5": c5}, default=float), flush=True)
        return

    wall0 = time.perf_counter()
    log("generating R-MAT scale 20")
    g = synth.rmat(20, 16, seed=20)
    sess = Session(0)
    G = sess.graph(g.off, g.nbr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = sess.tables(G, cv_seed=1)
    torch.cuda.synchronize()
    tables_s = time.perf_counter() - t0
    log(f"graph n={g.n} nnz={g.nnz} dmax={int(np.diff(g.off).max())}; tables {tables_s * 1e3:.1f} ms")
    pats = [synth.named_pattern(n) for n in PATTERNS]

    # the launch shape is tuned per pattern (the register-budget variant
    # that suits one pattern's paths can cost another's) and applied before
    # each of its estimates; it changes no result
    tuning = None
    pattern_tuning = {}
    if not args.no_tune:
        for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
            tun = sess.autotune(G, T, [p], args.tune_pilot, mode="switch", pattern_id=pid)
            pattern_tuning[name] = {"variant": tun.variant, "grab": tun.grab, "hub_window": tun.hub_window,
                                    "pilot_kernel_s": tun.seconds, "default_kernel_s": tun.default_seconds}
            log(f"tuned {name}: variant {tun.variant} grab {tun.grab} hub window {tun.hub_window} "
                f"({tun.default_seconds:.3f} s -> {tun.seconds:.3f} s)")
        # the legs after the steps keep the shape of the pattern that takes
        # most of a step
        tuning = dict(pattern_tuning["5-clique"], per_pattern=pattern_tuning)

    def apply_tuning(name):
        if name in pattern_tuning:
            t = pattern_tuning[name]
            sess.set_launch(True, 0, t["grab"], t["variant"], t["hub_window"])

    def restore_tuning():
        """Back to the headline's launch shape after a leg tuned its own."""
        apply_tuning("5-clique")

    n_step = -(-args.total_samples // args.steps)
    # what AUTO picks for estimates of n_step samples (the metering run must
    # take the same paths)
    rowtab = "on" if n_step >= 65536 else "off"

    def step(seed, first, walls=None):
        res = []
        for pid, p in enumerate(pats):
            t1 = time.perf_counter()
            apply_tuning(PATTERNS[pid])
            res.append(sess.estimate(G, T, p, n_step, seed, mode="switch", pattern_id=pid, first_sample=first))
            if walls is not None:
                walls[pid] += time.perf_counter() - t1
        return res

    for w in range(args.warmup):
        step(1000 + w, 0)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    walls = [0.0] * len(pats)
    for k in range(args.steps):
        results.append(step(7, k * n_step, walls))
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    restore_tuning()
    total = args.steps * len(pats) * n_step
    value = total / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"timed: {value:.4g} samples/s, {ms_per_step:.1f} ms/step")

    # the whole-range estimate per pattern, judged by exact counts where known
    exact = {"4-star": star_closed_form(g, 4)}
    gold = golden_cliques()
    if 5 in gold:
        exact["5-clique"] = gold[5]
    per_pattern = {}
    for pid, name in enumerate(PATTERNS):
        rs = [results[k][pid] for k in range(args.steps)]
        n, mean, var = merge_results(rs)
        ks = sum(r.sample_kernel_seconds for r in rs)
        entry = {"samples": int(n), "estimate": mean, "rel_var": var / max(mean * mean, 1e-300),
                 "std_err_rel": math.sqrt(var / n) / abs(mean) if n and mean else None,
                 "samples_per_s_kernel": n / ks if ks else None, "wall_s": walls[pid],
                 "kernel_s": ks, "launches": int(sum(r.sample_launches for r in rs)),
                 "tables_ms_per_estimate": 1e3 * float(np.mean([r.tables_seconds for r in rs]))}
        if name in exact:
            entry["exact"] = exact[name]
            entry["rel_err_vs_exact"] = (mean - exact[name]) / exact[name]
            entry["z_vs_exact"] = (mean - exact[name]) / math.sqrt(var / n) if var > 0 else None
        per_pattern[name] = entry
        log(f"{name}: estimate {mean:.6g} over {int(n)} samples"
            + (f", exact {exact[name]:.6g} (rel err {entry['rel_err_vs_exact']:.2e})" if name in exact else ""))

    # the clique on the degree-oriented graph, as the method runs cliques
    # (Sec. 5.4): the same steps with the 5-clique there instead
    value_dag = None
    dag = None
    if not args.skip_oriented:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        O = sess.orient(G)
        TO = sess.tables(O, cv_seed=1)
        torch.cuda.synchronize()
        orient_s = time.perf_counter() - t1
        cp = pats[PATTERNS.index("5-clique")]
        sess.estimate(O, TO, cp, n_step, 1000, mode="switch", pattern_id=0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dres = [sess.estimate(O, TO, cp, n_step, 7, mode="switch", pattern_id=0, first_sample=k * n_step)
                for k in range(args.steps)]
        torch.cuda.synchronize()
        dag_s = time.perf_counter() - t1
        n, mean, var = merge_results(dres)
        value_dag = total / (elapsed - walls[PATTERNS.index("5-clique")] + dag_s)
        dag = {"orient_and_tables_ms": 1e3 * orient_s, "nnz": O.nnz, "wall_s": dag_s, "estimate": mean,
               "rel_var": var / max(mean * mean, 1e-300), "value_with_clique_on_dag": value_dag}
        if "5-clique" in exact:
            dag["rel_err_vs_exact"] = (mean - exact["5-clique"]) / exact["5-clique"]
        log(f"5-clique on the degree DAG: {dag_s:.3f} s for the same samples; steps would run at "
            f"{value_dag:.4g} samples/s")
        TO.close()
        O.close()

    # ---- roofline of the sampling kernel -------------------------------
    log("roofline: metering sampled indices of the timed range")
    rng = np.random.Generator(np.random.PCG64(3))
    idx = np.sort(rng.choice(args.steps * n_step, size=min(args.meter_samples, args.steps * n_step), replace=False))
    meter = {}
    bytes_total = merge_total = 0.0
    kern_total = 0.0
    launches_total = 0
    hbm_total = 0.0
    # the lane sampler's launches (stars) are a kernel of their own
    lanes = {"bytes": 0.0, "kernel_s": 0.0, "launches": 0, "hbm": 0.0, "patterns": []}
    counters = None
    if os.path.exists(COUNTERS_FILE):
        c = json.load(open(COUNTERS_FILE))
        if c.get("kernel_source_sha") == kernel_source_hash():
            counters = c
    for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
        m = sess.meter(G, T, p, 7, idx, mode="switch", pattern_id=pid, rowtab=rowtab).astype(np.float64)
        rb, wb, segs, reqs = (float(x) for x in m.mean(axis=0))
        recs = sess.dump(G, T, p, 7, idx[: args.bytes_records], mode="switch", pattern_id=pid, rowtab=rowtab)
        mm = algorithmic_bytes(g, results[0][pid].plan, recs)
        e = per_pattern[name]
        nsamp = e["samples"]
        meter[name] = {"read_bytes_per_sample": rb, "write_bytes_per_sample": wb, "segments_per_sample": segs,
                       "requests_per_sample": reqs, "merge_model_bytes_per_sample": mm,
                       "achieved_gbs": (rb + wb) * nsamp / e["kernel_s"] / 1e9,
                       "segment_gbs": 64.0 * segs * nsamp / e["kernel_s"] / 1e9,
                       "merge_model_gbs": mm * nsamp / e["kernel_s"] / 1e9}
        meter[name]["kernel"] = "k_sample_lanes" if is_star(p) else "k_sample"
        hb = None
        if counters and name in counters.get("per_pattern", {}):
            hb = counters["per_pattern"][name]["hbm_bytes_per_sample"]
            meter[name]["traffic_gbs"] = hb * nsamp / e["kernel_s"] / 1e9
        if is_star(p):
            lanes["bytes"] += (rb + wb) * nsamp
            lanes["kernel_s"] += e["kernel_s"]
            lanes["launches"] += e["launches"]
            lanes["hbm"] += (hb or 0.0) * nsamp
            lanes["patterns"].append(name)
            continue
        bytes_total += (rb + wb) * nsamp
        merge_total += mm * nsamp
        kern_total += e["kernel_s"]
        launches_total += e["launches"]
        if hb is not None:
            hbm_total += hb * nsamp
    achieved = bytes_total / kern_total / 1e9
    # L2 hit rate of the k_sample dispatches (counter pass), weighted by time
    l2_hit = None
    if counters:
        num = den = 0.0
        for nm in PATTERNS:
            e = counters["per_pattern"].get(nm)
            if e and meter[nm]["kernel"] == "k_sample" and e.get("l2_hit_rate") is not None:
                num += e["l2_hit_rate"] * per_pattern[nm]["kernel_s"]
                den += per_pattern[nm]["kernel_s"]
        l2_hit = num / den if den else None
    seg_total = sum(meter[nm]["segments_per_sample"] * per_pattern[nm]["samples"] for nm in PATTERNS
                    if meter[nm]["kernel"] == "k_sample")
    bytes_per_segment = bytes_total / max(seg_total, 1.0)
    gather = None
    frac_gather = None
    s_match = None
    ceiling = None
    # the footprint the sampler gathers from: neighbour lists, offsets and
    # vertex records (the per-step tables are a few MB more)
    hot_bytes = 4 * g.nnz + 8 * (g.n + 1) + 16 * g.n
    footprint = "128MiB" if hot_bytes <= (256 << 20) else "8GiB"
    gather_peak = None
    if not args.skip_gather:
        wpc = 4 * (6 + (tuning["variant"] if tuning else 0))
        log(f"random-gather ceiling at {wpc} waves per CU")
        gather = gather_ceiling(sess, wpc)
        s_match = min(GATHER_SIZES, key=lambda s: abs(math.log2(s) - math.log2(max(bytes_per_segment, 1.0))))
        ceiling = gather[footprint][s_match]["dependent_gbs"]
        # request bytes over the ceiling of segments of the same mean size:
        # above 1 where the sampler's requests hit in L2 (reuse within a
        # sample), which the microbenchmark's random segments never do
        frac_gather = achieved / ceiling
        gather_peak = max(max(r["dependent_gbs"], r["independent_gbs"]) for r in gather[footprint].values())
        for label, rows in gather.items():
            for S, row in rows.items():
                log(f"  gather {label} {S:5d} B: dependent {row['dependent_gbs']:.0f} GB/s, independent "
                    f"{row['independent_gbs']:.0f} GB/s")
    roofline = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": (hbm_total / launches_total) if counters else None,
        "kernel": "k_sample", "avg_launch_ms": 1e3 * kern_total / launches_total,
        "algorithmic_bytes_per_launch": bytes_total / launches_total,
        "bytes_model": "request bytes counted per sample by the metering kernel (agis_meter_samples)",
        "segment_gbs": 64.0 * seg_total / kern_total / 1e9,
        "bytes_per_segment": bytes_per_segment,
        "gather_ceiling_gbs": ceiling,
        "gather_ceiling_segment_bytes": s_match,
        "gather_ceiling_footprint": footprint,
        "hot_bytes": hot_bytes,
        "requests_over_matched_gather_ceiling": frac_gather,
        "gather_peak_gbs": gather_peak,
        "traffic_frac": (hbm_total / kern_total / 1e9) / HBM_PEAK_GBS if counters else None,
        "traffic_frac_of_gather_peak": ((hbm_total / kern_total / 1e9) / gather_peak
                                        if counters and gather_peak else None),
        "merge_model_gbs": merge_total / kern_total / 1e9,
        "traffic_gbs": hbm_total / kern_total / 1e9 if counters else None,
        "traffic_source": os.path.relpath(COUNTERS_FILE, ROOT) if counters else None,
        "patterns": [nm for nm in PATTERNS if meter[nm]["kernel"] == "k_sample"],
        "l2_hit_rate": l2_hit,
    }
    if lanes["launches"]:
        la = lanes["bytes"] / lanes["kernel_s"] / 1e9
        roofline["lanes"] = {
            "kernel": "k_sample_lanes", "patterns": lanes["patterns"], "achieved": la, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": la / HBM_PEAK_GBS, "avg_launch_ms": 1e3 * lanes["kernel_s"] / lanes["launches"],
            "algorithmic_bytes_per_launch": lanes["bytes"] / lanes["launches"],
            "traffic": (lanes["hbm"] / lanes["launches"]) if counters and lanes["hbm"] else None}
    log(f"roofline: {achieved:.0f} GB/s of request bytes ({roofline['frac']:.3f} of HBM peak"
        + (f"; {frac_gather:.2f}x the {s_match}-B dependent-gather ceiling over {footprint}"
           if frac_gather else "") + ")"
        + (f"; HBM traffic {roofline['traffic_gbs']:.0f} GB/s ({roofline['traffic_frac']:.3f} of peak"
           + (f", {roofline['traffic_frac_of_gather_peak']:.3f} of the best gather rate" if gather_peak else "")
           + ")" if counters else "; no counters for these kernel sources"))

    detail = {"per_pattern": per_pattern, "meter": meter, "roofline": roofline, "gather": gather, "tuning": tuning,
              "dag": dag}

    learned = {}
    if not args.skip_learned and not args.skip_eps:
        learned = learned_four(args, sess, T, pats)
    eps_table = None
    if not args.skip_eps:
        eps_table = time_to_eps(args, sess, G, T, pats, learned)
        detail["time_to_1pct"] = eps_table
    if not args.skip_ablation:
        detail["term_ablation_and_beta"] = ablation_leg(args, sess, G, T)
    batch = None
    if not args.skip_batch:
        batch = batch_leg(args, sess, G, T, restore_tuning)
        detail["batch_32_patterns"] = batch
    if not args.skip_oriented:
        detail["cliques_oriented"] = oriented_leg(args, sess, G, T)
    if not args.skip_conc:
        detail["concentrations"] = conc_leg(args, sess, G, T)
    large = None
    if not args.skip_large:
        large = large_legs(args, sess, G, T, bpats_budgets(args), log, restore_tuning)
        detail["rmat24"] = large
    c1 = None
    c1_gpu = None
    if not (args.skip_c1 and args.skip_cpu):
        c1 = synth.chung_lu(n=10000, m=100000, seed=1)
    if not args.skip_c1:
        c1_gpu = c1_gpu_leg(sess, c1)
        detail["c1_gpu"] = c1_gpu
    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(g, c1, args.cpu_seconds)
        detail["cpu_baseline"] = cpu
        log(f"cpu baseline {cpu['value']:.4g} samples/s on {cpu['cores']} threads "
            f"({cpu['single_thread_value']:.4g} on one); C1 in full {cpu['c1_full']['seconds']:.1f} s")
        if c1_gpu:
            diffs = [abs(c1_gpu["runs"][k]["estimate"] - v["mean"]) / max(abs(v["mean"]), 1e-300)
                     for k, v in cpu["c1_full"]["runs"].items()]
            detail["c1_gpu_vs_oracle_max_rel_diff"] = max(diffs)
            log(f"C1: GPU vs oracle estimates, largest relative difference {max(diffs):.2e}")
        # the same R-MAT-20 sample indices on the GPU (the estimator's mean
        # over samples [0, n) of each pattern, as the oracle ran them)
        nr = cpu["rmat20_samples_per_pattern"]
        rd = []
        for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
            r = sess.estimate(G, T, p, nr, 7, mode="switch", pattern_id=pid, rowtab=rowtab)
            ref = cpu["rmat20_means"][name]
            rd.append(abs(r.estimate - ref) / max(abs(ref), 1e-300))
        cpu["rmat20_gpu_vs_oracle_max_rel_diff"] = max(rd)
        log(f"R-MAT-20: GPU vs oracle means over the first {nr} samples of each pattern, largest relative "
            f"difference {max(rd):.2e}")

    detail["wall_seconds"] = time.perf_counter() - wall0
    try:
        os.makedirs(os.path.dirname(args.detail), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(detail, f, indent=1, default=float)
        log(f"detail written to {args.detail}")
    except OSError as e:
        log(f"could not write the detail file: {e}")

    out = {
        "metric": "time to ±1% rel. err (95% CI) + samples/s: learned vs f_approx vs uniform",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"R-MAT scale 20 (ef 16, a=.57 b=.19 c=.19, seed 20) symmetric CSR; 5-clique, 5-cycle, "
                         f"house, 4-star; f_approx with switching (beta 4/5); {args.steps * n_step:.3g} samples per "
                         f"pattern ({n_step} per step)"),
            "n": g.n, "nnz": g.nnz, "samples_per_pattern": args.steps * n_step,
            "graph_tables_ms": round(1e3 * tables_s, 1),
        },
        "value_cliques_on_degree_dag": value_dag,
        "estimates": {k: {"estimate": v["estimate"], "rel_err_vs_exact": v.get("rel_err_vs_exact")}
                      for k, v in per_pattern.items()},
        "roofline": {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                              "avg_launch_ms", "traffic_gbs", "traffic_frac", "l2_hit_rate",
                                              "gather_ceiling_gbs", "gather_ceiling_segment_bytes",
                                              "requests_over_matched_gather_ceiling", "gather_peak_gbs",
                                              "traffic_frac_of_gather_peak", "gather_ceiling_footprint",
                                              "merge_model_gbs", "traffic_source")},
    }
    if "lanes" in roofline:
        out["roofline"]["lanes"] = {k: roofline["lanes"][k] for k in ("kernel", "patterns", "achieved", "frac",
                                                                       "avg_launch_ms", "traffic")}
    if eps_table:
        out["time_to_1pct_s"] = {
            name: {lab: round(eps_table[f"{name}/{lab}"]["seconds"], 5)
                   for lab in ("learned", "learned_with_fallback", "f_approx", "f_uniform")
                   if f"{name}/{lab}" in eps_table}
            for name in PATTERNS}
        out["samples_to_1pct"] = {
            name: {lab: eps_table[f"{name}/{lab}"]["samples"] for lab in ("learned", "f_approx", "f_uniform")
                   if f"{name}/{lab}" in eps_table}
            for name in PATTERNS}
    if batch:
        out["batch32_rmat20"] = {"seconds": round(batch["seconds"], 3), "samples_per_s": batch["samples_per_s"],
                                 "converged": batch["converged"],
                                 "one_at_a_time_seconds": round(batch["one_at_a_time_seconds"], 3)}
    if large:
        b = large["batch_32_patterns"]
        lp = large["learned_32_patterns"]
        out["rmat24"] = {"batch_seconds": round(b["seconds"], 3), "batch_converged": b["converged"],
                         "budget_scale": b["budget_scale"],
                         "learned_geomean_rel_var_vs_f_approx": lp["geomean_rel_var_learned_over_f_approx"],
                         "with_fallback": lp["geomean_rel_var_with_fallback_over_f_approx"]}
    if cpu:
        out["cpu_baseline"] = {"value": cpu["value"], "unit": cpu["unit"], "cores": cpu["cores"], "kind": "oracle",
                               "sample": cpu["sample"], "single_thread_value": cpu["single_thread_value"],
                               "gpu_vs_oracle_max_rel_diff": cpu.get("rmat20_gpu_vs_oracle_max_rel_diff"),
                               "c1_full_seconds": round(cpu["c1_full"]["seconds"], 2),
                               "host_model": cpu["host"]["model"], "nproc": cpu["host"]["nproc"]}
    out["detail"] = os.path.relpath(args.detail, ROOT)
    line = json.dumps(out)
    for drop in ("samples_to_1pct", "estimates", "rmat24", "batch32_rmat20"):
        if len(line) <= 4000:
            break
        out.pop(drop, None)
        line = json.dumps(out)
    T.close()
    G.close()
    sess.close()
    print(line, flush=True)


if __name__ == "__main__":
    main()
