"""Benchmark of the AGIS sampling estimator on one MI355X.

Workload: R-MAT scale 20 (2^20 vertices, edge factor 16, a=.57 b=.19 c=.19
d=.05, symmetrised, deduplicated, no self-loops; ~15.7M undirected edges),
patterns 5-clique, 5-cycle, house and 4-star, f_approx with the paper's
switching rule (beta = 4/5).  One step = one estimate per pattern over a
fixed batch of samples (first-step table build included, as the paper
counts it in mining time).  ``value`` is samples per second over the timed
steps.  Also reported: time to +-1% relative error at 95% confidence
(Algorithm 1) per pattern and proposal mode, the roofline of the sampling
kernel (random-gather bound: HBM), and the CPU oracle timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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
HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_sample_rmat20_counters.json")
KERNEL_SOURCES = ["paper_2601_01388_amd/csrc/kernels.hip", "paper_2601_01388_amd/csrc/agis_common.h"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


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


def is_clique(p) -> bool:
    return len(p.edges) == p.k * (p.k - 1) // 2


class HostCSR:
    def __init__(self, off, nbr):
        self.off = off
        self.nbr = nbr


def cpu_baseline(g, seconds_target: float):
    """The oracle (single thread) on a bounded sample of the same workload:
    the same patterns and mode, equal sample counts per pattern."""
    import oracle
    from oracle.pattern import compile_pattern
    import synth
    log("cpu baseline: oracle tables (setup, untimed)")
    t = oracle.Tables(g, cv_seed=1)
    og = ot = None
    samplers = []
    for name in PATTERNS:
        p = synth.named_pattern(name)
        cp = compile_pattern(p.k, p.edges, mode="switch")
        if is_clique(p):
            if og is None:
                og = oracle.orient(g)
                ot = oracle.Tables(og, cv_seed=1, adjacency=g)
            samplers.append(oracle.Sampler(og, ot, cp, seed=7, oriented=True))
        else:
            samplers.append(oracle.Sampler(g, t, cp, seed=7))
    # calibrate on a few samples, then size the timed sample
    per = []
    for s in samplers:
        t0 = time.perf_counter()
        s.run(0, 200)
        per.append((time.perf_counter() - t0) / 200)
    n_each = max(200, int(seconds_target / max(sum(per), 1e-9)))
    log(f"cpu baseline: {n_each} samples per pattern")
    t0 = time.perf_counter()
    for s in samplers:
        s.run(0, n_each)
    el = time.perf_counter() - t0
    return {
        "value": len(PATTERNS) * n_each / el,
        "unit": "samples/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {n_each} sample indices of each of {', '.join(PATTERNS)} (f_approx+switch, seed 7, "
                  f"cliques on the degree-oriented graph) on the same R-MAT-20 graph, single-threaded C oracle, "
                  f"{el:.1f} s",
        "host": platform.processor() or platform.machine(),
        "host_threads_available": os.cpu_count(),
    }


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=1 << 22, help="samples per pattern per step")
    ap.add_argument("--eps-budget", type=int, default=10 ** 8, help="sample budget of each run to +-1%%")
    ap.add_argument("--skip-eps", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--bytes-records", type=int, default=1500)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run 3 plain device copies of this many bytes (counter calibration) and exit")
    ap.add_argument("--tune-pilot", type=int, default=1 << 20, help="pilot samples per pattern of the autotuner")
    ap.add_argument("--batch-tune-pilot", type=int, default=1 << 15,
                    help="pilot samples per pattern of the batch legs' autotuning")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
    ap.add_argument("--skip-ablation", action="store_true")
    ap.add_argument("--skip-conc", action="store_true")
    ap.add_argument("--skip-oriented", action="store_true")
    ap.add_argument("--conc-budget", type=int, default=20_000_000,
                    help="sample budget per pattern of the concentration runs (to +-1%%)")
    ap.add_argument("--skip-large", action="store_true",
                    help="skip the R-MAT scale 24 legs (32-pattern batch; learned proposal trained on scale 20)")
    ap.add_argument("--large-budget-scale", type=float, default=0.1,
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
    # cliques run on the degree-oriented graph, as the method does for them
    # (Sec. 5.4); it is built once per graph with its tables, like the
    # symmetric graph's tables (preprocessing, outside the timed steps)
    O = TO = None
    orient_s = 0.0
    if any(is_clique(p) for p in pats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        O = sess.orient(G)
        TO = sess.tables(O, cv_seed=1)
        torch.cuda.synchronize()
        orient_s = time.perf_counter() - t0
        log(f"degree-oriented graph for the cliques: nnz={O.nnz}, orientation and tables {orient_s * 1e3:.1f} ms")

    def graph_of(p):
        return (O, TO) if is_clique(p) else (G, T)

    tuning = None
    if not args.no_tune:
        # tuned on the patterns that run on the symmetric graph (the
        # launch shape is one per context)
        tpats = [p for p in pats if not is_clique(p)] or pats
        log(f"autotuning the sampler launch on {len(tpats)} patterns")
        tun = sess.autotune(G, T, tpats, args.tune_pilot, mode="switch")
        tuning = {"variant": tun.variant, "grab": tun.grab, "hub_window": tun.hub_window, "pilot_kernel_s": tun.seconds,
                  "default_kernel_s": tun.default_seconds}
        log(f"tuned: variant {tun.variant} grab {tun.grab} hub window {tun.hub_window} "
            f"({tun.default_seconds:.3f} s -> {tun.seconds:.3f} s)")

    def restore_tuning():
        """Back to the headline's launch shape after a leg tuned its own."""
        if tuning is not None:
            sess.set_launch(True, 0, tuning["grab"], tuning["variant"], tuning["hub_window"])

    def step(seed, walls=None):
        res = []
        for pid, p in enumerate(pats):
            t1 = time.perf_counter()
            gg, tt = graph_of(p)
            res.append(sess.estimate(gg, tt, p, args.samples, seed, mode="switch", pattern_id=pid))
            if walls is not None:
                walls[pid] += time.perf_counter() - t1
        return res

    # the timed steps' clique estimates on the symmetric graph instead, for
    # comparison (not the headline): their wall time replaces the oriented
    # ones' (run first, so that the timed launches are the last ones)
    sym_s = 0.0
    if O is not None:
        for pid, p in enumerate(pats):
            if is_clique(p):
                sess.estimate(G, T, p, args.samples, 999, mode="switch", pattern_id=pid)  # warmup
        for k in range(args.steps):
            for pid, p in enumerate(pats):
                if is_clique(p):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    sess.estimate(G, T, p, args.samples, 7 + k, mode="switch", pattern_id=pid)
                    sym_s += time.perf_counter() - t1
    for w in range(args.warmup):
        step(1000 + w)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    walls = [0.0] * len(pats)
    for k in range(args.steps):
        results.append(step(7 + k, walls))
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value_symmetric = None
    if O is not None:
        clique_s = sum(w for w, p in zip(walls, pats) if is_clique(p))
        value_symmetric = args.steps * len(pats) * args.samples / (elapsed - clique_s + sym_s)
    total_samples = args.steps * len(pats) * args.samples
    value = total_samples / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    kern_s = sum(r.sample_kernel_seconds for rs in results for r in rs)
    launches = sum(r.sample_launches for rs in results for r in rs)
    per_pattern = {}
    for pid, name in enumerate(PATTERNS):
        ks = sum(rs[pid].sample_kernel_seconds for rs in results)
        per_pattern[name] = {
            "graph": "degree-oriented" if is_clique(pats[pid]) else "symmetric",
            "samples_per_s_kernel": args.steps * args.samples / ks,
            "estimate": results[-1][pid].estimate,
            "rel_var": results[-1][pid].variance / max(results[-1][pid].estimate ** 2, 1e-300),
            "tables_ms": 1e3 * results[-1][pid].tables_seconds,
        }
    log(f"timed: {value:.4g} samples/s, {ms_per_step:.1f} ms/step"
        + (f"; cliques on the symmetric graph instead: {value_symmetric:.4g} samples/s" if value_symmetric else ""))

    # algorithmic bytes per sample, from dumped records of the timed stream
    log("algorithmic bytes from sampled records")
    bytes_per_sample = {}
    rng = np.random.Generator(np.random.PCG64(3))
    idx = np.sort(rng.integers(0, args.samples, size=args.bytes_records, dtype=np.uint64))
    host_dag = None
    for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
        gg, tt = graph_of(p)
        recs = sess.dump(gg, tt, p, 7, idx, mode="switch", pattern_id=pid)
        hg = g
        if gg is O:
            if host_dag is None:
                host_dag = HostCSR(*O.csr())
            hg = host_dag
        bytes_per_sample[name] = algorithmic_bytes(hg, results[0][pid].plan, recs)
    # dominant kernel: the sampling kernel; bytes per launch = samples per
    # launch x mean bytes per sample (equal sample counts per pattern)
    mean_bytes = float(np.mean([bytes_per_sample[n] for n in PATTERNS]))
    avg_launch_s = kern_s / launches
    achieved_gbs = mean_bytes * args.samples / avg_launch_s / 1e9
    # HBM traffic per launch from the committed FETCH_SIZE / WRITE_SIZE
    # counter runs (calibrated on a plain copy), valid only while the kernel
    # sources are the ones the counters were taken with; the counters give
    # bytes per sample (mean over the four patterns), scaled to this launch
    traffic = None
    l2_hit = None
    if os.path.exists(COUNTERS_FILE):
        c = json.load(open(COUNTERS_FILE))
        if c.get("kernel_source_sha") == kernel_source_hash():
            traffic = c["hbm_bytes_per_sample_mean"] * args.samples
            rates = [v.get("l2_hit_rate") for v in c["per_pattern"].values()]
            if all(r is not None for r in rates):
                l2_hit = {k: v["l2_hit_rate"] for k, v in c["per_pattern"].items()}
    roofline = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_sample", "avg_launch_ms": 1e3 * avg_launch_s,
                "algorithmic_bytes_per_launch": mean_bytes * args.samples,
                "algorithmic_bytes_per_sample": bytes_per_sample,
                "traffic_gbs": (traffic / avg_launch_s / 1e9) if traffic else None,
                "l2_hit_rate": l2_hit}

    # learned proposal: one MLP per pattern, trained on extension counts the
    # sampler produces on a smaller R-MAT graph (scale 18, seed 18), then
    # BF16 inference into pick tables for this graph
    learned = {}
    if not args.skip_learned and not args.skip_eps:
        from paper_2601_01388_amd.session import mlp_init
        log("learned proposal: training graph R-MAT scale 18")
        gtr = synth.rmat(18, 16, seed=18)
        Gtr = sess.graph(gtr.off, gtr.nbr)
        Ttr = sess.tables(Gtr, cv_seed=1)
        ftr = sess.features(Ttr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fev = sess.features(T)
        torch.cuda.synchronize()
        feat_s = time.perf_counter() - t0
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
            init = mlp_init(7 + pid, float(np.average(tg, weights=wt)) if rows["rows"] else 0.0,
                            zero_output=residual)
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

    # time to +-1% (95% CI) per pattern and proposal mode
    eps_table = {}
    if not args.skip_eps:
        for pid, (name, p) in enumerate(zip(PATTERNS, pats)):
            for mode in ("learned", "switch", "always", "uniform"):
                if mode == "learned" and name not in learned:
                    continue
                kw = dict(learned=learned[name]["ptrs"]) if mode == "learned" else {}
                r = sess.estimate(G, T, p, args.eps_budget, 11, mode=mode, pattern_id=pid, eps=0.01, delta=0.05,
                                  check_every=1 << 16, min_samples=1 << 14, **kw)
                need = r.n * (r.eps_hat / 0.01) ** 2 if math.isfinite(r.eps_hat) else None
                label = {"switch": "f_approx", "always": "f_approx_always", "uniform": "f_uniform",
                         "learned": "learned"}[mode]
                entry = {
                    "seconds": r.seconds, "converged": bool(r.converged), "samples": r.n, "estimate": r.estimate,
                    "eps_hat": r.eps_hat, "rel_var": r.variance / max(r.estimate ** 2, 1e-300),
                    "samples_needed": need,
                }
                if mode == "learned":
                    entry["seconds_incl_table_inference"] = r.seconds + learned[name]["info"]["infer_seconds"]
                    entry.update(learned[name]["info"])
                eps_table[f"{name}/{label}"] = entry
                log(f"+-1% {name} {label}: {r.seconds:.3f} s, n={r.n}, rel.var {entry['rel_var']:.4g}, "
                    f"converged={bool(r.converged)}")
        for pid, name in enumerate(PATTERNS):
            if f"{name}/learned" not in eps_table:
                continue
            eps_table[f"{name}/learned"]["rel_var_vs_f_approx"] = (
                eps_table[f"{name}/learned"]["rel_var"] / max(eps_table[f"{name}/f_approx"]["rel_var"], 1e-300))
            # fallback: a pilot of each proposal on fresh samples keeps the
            # learned tables only if their variance per sample is lower
            t0 = time.perf_counter()
            pl = sess.estimate(G, T, pats[pid], args.pilot_samples, 97, mode="learned", pattern_id=pid,
                               learned=learned[name]["ptrs"])
            pa = sess.estimate(G, T, pats[pid], args.pilot_samples, 97, mode="switch", pattern_id=pid)
            pilot_s = time.perf_counter() - t0
            keep = pl.variance / max(pl.estimate ** 2, 1e-300) < pa.variance / max(pa.estimate ** 2, 1e-300)
            chosen = eps_table[f"{name}/learned" if keep else f"{name}/f_approx"]
            eps_table[f"{name}/learned_with_fallback"] = {
                "chosen": "learned" if keep else "f_approx", "pilot_seconds": pilot_s,
                "seconds": chosen["seconds"] + pilot_s, "samples": chosen["samples"],
                "converged": chosen["converged"], "estimate": chosen["estimate"], "rel_var": chosen["rel_var"]}
            log(f"{name}: pilot keeps {'learned' if keep else 'f_approx'}")

    # incremental terms of f_approx (T[F1]; T[F1] T[I1]; all three) and the
    # switching threshold beta, as in the paper's analysis of the
    # approximation and of beta: variance per sample and the samples
    # Algorithm 1 needs for +-1% at 95% (z^2 rel.var / eps^2)
    ablation = None
    if not args.skip_ablation:
        z2 = 1.959963984540054 ** 2
        ablation = {"samples": args.ablation_samples, "terms": {}, "beta": {}}
        t0 = time.perf_counter()
        for name in ["4-clique", "4-path", "5-clique", "5-cycle", "house"]:
            p = synth.named_pattern(name)
            row = {}
            for terms in ("f1", "f1_i1", "all"):
                r = sess.estimate(G, T, p, args.ablation_samples, 17, mode="switch", terms=terms)
                rv = r.variance / max(r.estimate ** 2, 1e-300)
                row[terms] = {"rel_var": rv, "samples_needed": z2 * rv / 1e-4, "estimate": r.estimate,
                              "seconds_per_sample": r.seconds / r.n}
            ablation["terms"][name] = row
        betas = [("-inf", (-1, 0)), ("1/2", (1, 2)), ("4/5", (4, 5)), ("5/6", (5, 6)), ("1", (1, 1)),
                 ("+inf", (1, 0))]
        for name in ["house", "5-cycle", "6-cycle", "chordal-7-cycle"]:
            p = synth.named_pattern(name)
            row = {}
            for label, beta in betas:
                r = sess.estimate(G, T, p, args.ablation_samples, 19, mode="switch", beta=beta)
                rv = r.variance / max(r.estimate ** 2, 1e-300)
                row[label] = {"rel_var": rv, "samples_needed": z2 * rv / 1e-4, "estimate": r.estimate,
                              "seconds_per_sample": r.seconds / r.n,
                              "uniform_steps": int(sum(1 for i in range(p.k) if not r.plan.decision[i]))}
            ablation["beta"][name] = row
        ablation["seconds"] = time.perf_counter() - t0
        log(f"term ablation and beta sweep: {ablation['seconds']:.1f} s")
        for name, row in ablation["terms"].items():
            log("  terms " + name + ": " + ", ".join(f"{k} {v['rel_var']:.3g}" for k, v in row.items()))
        for name, row in ablation["beta"].items():
            log("  beta " + name + ": " + ", ".join(f"{k} {v['rel_var']:.3g}" for k, v in row.items()))

    # 32 connected patterns of 4-7 vertices (seed 3) with uneven budgets,
    # all run to +-1% in one batch of rounds (each a persistent launch)
    batch = None
    if not args.skip_batch:
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
        restore_tuning()
        batch = {
            "patterns": 32, "tuning": btune, "seconds": bt, "samples": int(sum(r.n for r in res)),
            "converged": int(sum(r.converged for r in res)),
            "samples_per_s": sum(r.n for r in res) / bt,
            "budget_total": int(sum(budgets)),
            "per_pattern": [{"k": p.k, "edges": len(p.edges), "budget": b, "samples": r.n,
                             "converged": bool(r.converged), "seconds": r.seconds,
                             "rel_var": r.variance / max(r.estimate ** 2, 1e-300)}
                            for p, b, r in zip(bpats, budgets, res)],
        }
        log(f"batch: {bt:.2f} s, {batch['converged']}/32 converged, {batch['samples']:.3g} samples")

    # cliques on the degree-oriented graph (each clique one trajectory) vs
    # the symmetric graph: samples/s, variance per sample, time to +-1%
    oriented = None
    if not args.skip_oriented:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        O = sess.orient(G)
        TO = sess.tables(O, cv_seed=1)
        torch.cuda.synchronize()
        oriented = {"orient_and_tables_ms": 1e3 * (time.perf_counter() - t0), "nnz": O.nnz, "patterns": {}}
        for k in (4, 5):
            p = synth.patterns.clique(k)
            row = {}
            for label, (gg, tt) in (("oriented", (O, TO)), ("symmetric", (G, T))):
                r = sess.estimate(gg, tt, p, args.samples, 29, mode="switch", pattern_id=k)
                e = sess.estimate(gg, tt, p, args.eps_budget, 31, mode="switch", pattern_id=k, eps=0.01, delta=0.05,
                                  check_every=1 << 16, min_samples=1 << 14)
                row[label] = {"samples_per_s_kernel": r.n / max(r.sample_kernel_seconds, 1e-12),
                              "rel_var": r.variance / max(r.estimate ** 2, 1e-300), "estimate": r.estimate,
                              "time_to_1pct_s": e.seconds, "samples_to_1pct": e.n, "converged": bool(e.converged)}
            oriented["patterns"][f"{k}-clique"] = row
            log(f"{k}-clique oriented: {row['oriented']['samples_per_s_kernel']:.3g} samples/s, rel.var "
                f"{row['oriented']['rel_var']:.3g}, +-1% in {row['oriented']['time_to_1pct_s']:.4f} s; symmetric: "
                f"{row['symmetric']['samples_per_s_kernel']:.3g} samples/s, rel.var {row['symmetric']['rel_var']:.3g}, "
                f"+-1% in {row['symmetric']['time_to_1pct_s']:.4f} s")
        TO.close()
        O.close()

    # concentrations of all connected 4- and 5-vertex patterns (6 and 21),
    # each pattern run to +-1% inside batched launches, as in the paper's
    # comparison with MCMC estimators
    concentration = None
    if not args.skip_conc:
        concentration = {}
        for k in (4, 5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = sess.concentrations(G, T, k, args.conc_budget, 23, mode="switch", eps=0.01, delta=0.05,
                                      check_every=1 << 16, min_samples=1 << 14)
            torch.cuda.synchronize()
            ct = time.perf_counter() - t0
            res = out["results"]
            concentration[f"k{k}"] = {
                "patterns": len(res), "seconds": ct, "budget_per_pattern": args.conc_budget,
                "converged": int(sum(r.converged for r in res)), "samples": int(sum(r.n for r in res)),
                "per_pattern": [{"edges": [list(e) for e in p[1]], "copies": r.copies, "eps_hat": r.eps_hat,
                                 "conc_edge": float(ce), "conc_induced": float(ci), "induced": float(ind)}
                                for p, r, ce, ci, ind in zip(out["patterns"], res, out["conc_edge"],
                                                              out["conc_induced"], out["induced"])]}
            log(f"concentrations k={k}: {len(res)} patterns, {concentration[f'k{k}']['converged']} converged, "
                f"{ct:.2f} s")

    # R-MAT scale 24 (generated on the GPU): the 32-pattern batch run to
    # +-1%, and the learned proposal trained on extension counts of the
    # scale-20 graph, evaluated against f_approx for variance per sample
    large = None
    if not args.skip_large:
        large = large_legs(args, sess, G, T, bpats_budgets(args), log, restore_tuning)

    cpu = None
    if not args.skip_cpu:
        cpu = cpu_baseline(g, args.cpu_seconds)
        log(f"cpu baseline {cpu['value']:.4g} samples/s")

    out = {
        "metric": "time to ±1% rel. err (95% CI) + samples/s: learned vs f_approx vs uniform",
        "value": value,
        "value_cliques_on_symmetric_graph": value_symmetric,
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
            "workload": "R-MAT scale 20 (ef 16, a=.57 b=.19 c=.19), patterns 5-clique/5-cycle/house/4-star, "
                        "f_approx with switching (beta=4/5); the clique on the degree-oriented graph (Sec. 5.4)",
            "orientation_and_tables_ms": 1e3 * orient_s,
            "samples_per_pattern_per_step": args.samples,
            "graph": {"n": g.n, "nnz": g.nnz, "seed": 20},
            "tables_ms": 1e3 * tables_s,
        },
        "tuning": tuning,
        "per_pattern": per_pattern,
        "batch_32_patterns": batch,
        "rmat24": large,
        "concentrations": concentration,
        "cliques_oriented": oriented,
        "term_ablation_and_beta": ablation,
        "time_to_1pct": eps_table,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": {
            "hardware": "AMD Ryzen Threadripper PRO 7985WX, 48 cores (C++/OpenMP, one sampler per thread)",
            "graphs": "real graphs (LiveJournal to GSH-2015), eps = 0.1, delta = 0.01",
            "geomean_speedup_vs_scalegpm": 28.5,
            "geomean_speedup_vs_peregrine": 63108,
            "note": "context only: the paper reports no samples/s and no GPU figure",
        },
    }
    print(json.dumps(out), flush=True)
    T.close()
    G.close()
    sess.close()


if __name__ == "__main__":
    main()
