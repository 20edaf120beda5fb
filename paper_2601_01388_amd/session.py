"""Convenience layer over the C names: owns torch device buffers for a CSR
graph and keeps the handles alive.  Still argument marshalling only; the
estimator runs in libagis.so."""

from __future__ import annotations

import ctypes

import numpy as np

from . import (AGIS_CSR_VALIDATE, LC_MIN_DEFAULT, RECORD_DTYPE, RECORD_BYTES, agis_build_proposal_tables,
               agis_autotune, agis_compile_pattern, agis_concentrations, agis_connected_patterns, agis_step1_weights,
               agis_orient,
               agis_graph_export, agis_create, agis_destroy, agis_dump_samples, agis_estimate, agis_release_scratch,
               agis_estimate_batch, agis_features, agis_graph_destroy, agis_learn_rows, agis_learn_targets,
               agis_load_csr, agis_mlp_grad, agis_mlp_infer, agis_mlp_param_count, agis_mlp_train, agis_set_launch,
               agis_step_log_weights, agis_meter_samples, agis_gather_bench,
               agis_tables_destroy, agis_tables_export, make_params, make_pattern, lib)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the AGIS library needs a ROCm GPU; none is visible")
    return torch


class Graph:
    """A CSR graph on the device: host numpy arrays (uint64 off, uint32 nbr)
    are copied; device tensors (int64 off, int32 nbr on the session's GPU)
    are used in place."""

    def __init__(self, sess, off, nbr, validate: bool = True):
        torch = _torch()
        self.sess = sess
        self.n = int(off.shape[0] - 1)
        self.nnz = int(nbr.shape[0])
        dev = sess.device
        if isinstance(off, torch.Tensor):
            if off.dtype != torch.int64 or nbr.dtype != torch.int32 or off.device != dev or nbr.device != dev:
                raise ValueError("device CSR must be int64 offsets and int32 neighbours on the session's GPU")
            self.d_off = off.contiguous()
            self.d_nbr = nbr.contiguous() if self.nnz else torch.zeros(1, dtype=torch.int32, device=dev)
        else:
            self.d_off = torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).to(dev)
            nb = np.ascontiguousarray(nbr, dtype=np.uint32).view(np.int32)
            self.d_nbr = torch.from_numpy(nb if nb.size else np.zeros(1, dtype=np.int32)).to(dev)
        self.handle = agis_load_csr(sess.ctx, self.d_off.data_ptr(), self.d_nbr.data_ptr(), self.n, self.nnz,
                                    AGIS_CSR_VALIDATE if validate else 0)

    def close(self):
        if self.handle:
            agis_graph_destroy(self.handle)
            self.handle = None


class _DeviceArray:
    """A library-owned device buffer seen by torch (no copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 3}


class OrientedGraph:
    """The degree orientation of a Graph (agis_orient), owned by the library;
    keeps its undirected graph alive."""

    def __init__(self, sess, graph: Graph):
        self.sess = sess
        self.parent = graph
        self.handle = agis_orient(sess.ctx, graph.handle)
        self.n, self.nnz, self._off, self._nbr = agis_graph_export(sess.ctx, self.handle)

    def csr(self):
        """(off uint64, nbr uint32) host copies of the oriented CSR."""
        torch = _torch()
        off = torch.as_tensor(_DeviceArray(self._off, self.n + 1, "<i8"), device=self.sess.device)
        o = off.cpu().numpy().view(np.uint64).copy()
        if not self.nnz:
            return o, np.zeros(0, dtype=np.uint32)
        nbr = torch.as_tensor(_DeviceArray(self._nbr, self.nnz, "<i4"), device=self.sess.device)
        return o, nbr.cpu().numpy().view(np.uint32).copy()

    def close(self):
        if self.handle:
            agis_graph_destroy(self.handle)
            self.handle = None


class Tables:
    def __init__(self, sess, graph: Graph, cv_seed: int = 0, lc_min: int = LC_MIN_DEFAULT, exact_cv: bool = False):
        self.sess = sess
        self.graph = graph
        self.handle = agis_build_proposal_tables(sess.ctx, graph.handle, cv_seed, lc_min, exact_cv)

    def export(self) -> dict:
        torch = _torch()
        n = self.graph.n
        dev = self.sess.device
        deg = torch.zeros(n, dtype=torch.int32, device=dev)
        s2 = torch.zeros(n, dtype=torch.int64, device=dev)
        hits = torch.zeros(n, dtype=torch.int64, device=dev)
        trials = torch.zeros(n, dtype=torch.int64, device=dev)
        la = torch.zeros(n, dtype=torch.int32, device=dev)
        lc = torch.zeros(n, dtype=torch.int32, device=dev)
        agis_tables_export(self.sess.ctx, self.handle, deg.data_ptr(), s2.data_ptr(), hits.data_ptr(),
                           trials.data_ptr(), la.data_ptr(), lc.data_ptr())
        return {
            "deg": deg.cpu().numpy().view(np.uint32), "s2": s2.cpu().numpy().view(np.uint64),
            "hits": hits.cpu().numpy().view(np.uint64), "trials": trials.cpu().numpy().view(np.uint64),
            "la": la.cpu().numpy(), "lc": lc.cpu().numpy(),
        }

    def close(self):
        if self.handle:
            agis_tables_destroy(self.handle)
            self.handle = None


class Session:
    """One library context on one GPU, on torch's current stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        lib()
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = agis_create(device, self.stream.cuda_stream)

    def graph(self, off, nbr, validate=True) -> Graph:
        return Graph(self, off, nbr, validate)

    def orient(self, graph: Graph) -> OrientedGraph:
        return OrientedGraph(self, graph)

    def tables(self, graph: Graph, cv_seed=0, lc_min=LC_MIN_DEFAULT, exact_cv=False) -> Tables:
        return Tables(self, graph, cv_seed, lc_min, exact_cv)

    def estimate(self, graph: Graph, tables: Tables, pattern, n_samples: int, seed: int, order=None, **kw):
        p = make_pattern(pattern.k, pattern.adj8())
        return agis_estimate(self.ctx, graph.handle, tables.handle, p, n_samples, seed, make_params(**kw), order=order)

    def estimate_batch(self, graph: Graph, tables: Tables, patterns, budgets, seed: int, **kw):
        ps = [make_pattern(p.k, p.adj8()) for p in patterns]
        return agis_estimate_batch(self.ctx, graph.handle, tables.handle, ps, [int(b) for b in budgets], seed,
                                   make_params(**kw))

    def autotune(self, graph: Graph, tables: Tables, patterns, pilot_samples: int, **kw):
        ps = [make_pattern(p.k, p.adj8()) for p in patterns]
        return agis_autotune(self.ctx, graph.handle, tables.handle, ps, pilot_samples, make_params(**kw))

    def step1_weights(self, graph: Graph, tables: Tables, pattern, order=None, **kw):
        """(q1 int64 host array, total): the first-step proposal q1[v] / total."""
        torch = _torch()
        q1 = torch.zeros(max(graph.n, 1), dtype=torch.int32, device=self.device)
        total = agis_step1_weights(self.ctx, graph.handle, tables.handle, make_pattern(pattern.k, pattern.adj8()),
                                   make_params(**kw), q1.data_ptr(), order=order)
        return q1.cpu().numpy()[: graph.n].view(np.uint32).astype(np.int64), total

    def concentrations(self, graph: Graph, tables: Tables, k: int, budget: int, seed: int, **kw):
        """Estimates every connected k-vertex pattern (agis_connected_patterns;
        batched launches of at most 64 patterns) and returns their
        concentrations: edge-induced (copies / total) and vertex-induced
        (agis_concentrations).  patterns: (k, edges) per pattern."""
        pats = agis_connected_patterns(k)
        res = []
        for lo in range(0, len(pats), 64):
            chunk = pats[lo:lo + 64]
            res += agis_estimate_batch(self.ctx, graph.handle, tables.handle, chunk, [int(budget)] * len(chunk), seed,
                                       make_params(**dict(kw, pattern_id=kw.get("pattern_id", 0) + lo)))
        ce, ind, ci = agis_concentrations(pats, [r.copies for r in res])
        edges = [(p.k, [(a, b) for a in range(p.k) for b in range(a + 1, p.k) if p.adj[a] >> b & 1]) for p in pats]
        return {"patterns": edges, "results": res, "conc_edge": ce, "induced": ind, "conc_induced": ci}

    def set_launch(self, use_graphs=True, blocks_per_cu=0, grab=0, variant=0, hub_window=0):
        agis_set_launch(self.ctx, use_graphs, blocks_per_cu, grab, variant, hub_window)

    def dump(self, graph: Graph, tables: Tables, pattern, seed: int, indices, order=None, **kw) -> np.ndarray:
        torch = _torch()
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        m = idx.size
        d_idx = torch.from_numpy(idx.view(np.int64) if m else np.zeros(1, dtype=np.int64)).to(self.device)
        d_out = torch.zeros(max(m, 1) * RECORD_BYTES, dtype=torch.uint8, device=self.device)
        p = make_pattern(pattern.k, pattern.adj8())
        agis_dump_samples(self.ctx, graph.handle, tables.handle, p, seed, make_params(**kw), d_idx.data_ptr(), m,
                          d_out.data_ptr(), order=order)
        return d_out.cpu().numpy()[: m * RECORD_BYTES].view(RECORD_DTYPE).copy()

    def meter(self, graph: Graph, tables: Tables, pattern, seed: int, indices, order=None, **kw) -> np.ndarray:
        """Per sample (rows of the index list): read bytes, written bytes,
        64-byte segments and wave-level requests of the production paths
        (agis_meter_samples), as a uint64 array of shape (m, 4)."""
        torch = _torch()
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        m = idx.size
        d_idx = torch.from_numpy(idx.view(np.int64) if m else np.zeros(1, dtype=np.int64)).to(self.device)
        d_out = torch.zeros(max(m, 1) * 4, dtype=torch.int64, device=self.device)
        p = make_pattern(pattern.k, pattern.adj8())
        agis_meter_samples(self.ctx, graph.handle, tables.handle, p, seed, make_params(**kw), d_idx.data_ptr(), m,
                           d_out.data_ptr(), order=order)
        return d_out.cpu().numpy()[: m * 4].view(np.uint64).reshape(m, 4).copy()

    def gather_bench(self, buf, seg_bytes: int, dependent: bool, waves_per_cu: int = 28, rounds: int = 64,
                     seed: int = 1):
        """(seconds, useful bytes) of one random-gather run over the device
        tensor buf (agis_gather_bench)."""
        torch = _torch()
        sink = torch.zeros(1024, dtype=torch.int64, device=self.device)
        return agis_gather_bench(self.ctx, buf.data_ptr(), buf.numel() * buf.element_size(), seg_bytes, dependent,
                                 waves_per_cu, rounds, seed, sink.data_ptr())

    # ---------------------------------------------------------------- learned proposal

    def features(self, tables: Tables):
        torch = _torch()
        f = torch.zeros((tables.graph.n, 4), dtype=torch.float32, device=self.device)
        agis_features(self.ctx, tables.handle, f.data_ptr())
        return f

    def learn_targets(self, graph: Graph, tables: Tables, pattern, n_samples: int, seed: int, **kw):
        torch = _torch()
        k, n = pattern.k, graph.n
        sums = torch.zeros((k, n), dtype=torch.float64, device=self.device)
        counts = torch.zeros((k, n), dtype=torch.int32, device=self.device)
        p = make_pattern(pattern.k, pattern.adj8())
        agis_learn_targets(self.ctx, graph.handle, tables.handle, p, n_samples, seed, make_params(**kw),
                           sums.data_ptr(), counts.data_ptr())
        return sums, counts

    def step_log_weights(self, tables: Tables, pattern, mode="learned"):
        """f_approx Q16 log weights of every vertex, one row per step of the
        pattern's plan (rows of steps that are not weighted stay zero)."""
        torch = _torch()
        plan = agis_compile_pattern(make_pattern(pattern.k, pattern.adj8()), params=make_params(mode=mode))
        base = torch.zeros((pattern.k, tables.graph.n), dtype=torch.int32, device=self.device)
        for i in range(pattern.k):
            if plan.decision[i] and plan.f1[i] > 0:
                agis_step_log_weights(self.ctx, tables.handle, plan.b[i], plan.f1[i], plan.ie[i], plan.f2[i],
                                      base[i].data_ptr())
        return base

    def learn_rows(self, sums, counts, step_mask: int, min_count: int = 2, base=None):
        torch = _torch()
        k, n = sums.shape
        cap = max(k * n, 1)
        vtx = torch.zeros(cap, dtype=torch.int32, device=self.device)
        cls = torch.zeros(cap, dtype=torch.uint8, device=self.device)
        tgt = torch.zeros(cap, dtype=torch.float32, device=self.device)
        wt = torch.zeros(cap, dtype=torch.float32, device=self.device)
        rows = agis_learn_rows(self.ctx, sums.data_ptr(), counts.data_ptr(), k, n, step_mask, min_count,
                               vtx.data_ptr(), cls.data_ptr(), tgt.data_ptr(), wt.data_ptr(),
                               base.data_ptr() if base is not None else 0)
        return {"vtx": vtx[:rows], "cls": cls[:rows], "target": tgt[:rows], "weight": wt[:rows], "rows": rows}

    def mlp_grad(self, params, feats, rows: dict):
        torch = _torch()
        grad = torch.zeros(agis_mlp_param_count(), dtype=torch.float32, device=self.device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        wsum = float(rows["weight"].double().sum().item())
        agis_mlp_grad(self.ctx, params.data_ptr(), feats.data_ptr(), rows["vtx"].data_ptr(), rows["cls"].data_ptr(),
                      rows["target"].data_ptr(), rows["weight"].data_ptr(), rows["rows"], wsum, grad.data_ptr(),
                      loss.data_ptr())
        return grad, float(loss.item())

    def mlp_train(self, params, feats, rows: dict, epochs: int, batch: int, lr: float, seed: int):
        return agis_mlp_train(self.ctx, params.data_ptr(), feats.data_ptr(), rows["vtx"].data_ptr(),
                              rows["cls"].data_ptr(), rows["target"].data_ptr(), rows["weight"].data_ptr(),
                              rows["rows"], epochs, batch, lr, seed)

    def mlp_infer(self, params, feats, position_class: int, want_y: bool = False, base=None, y_range=None):
        torch = _torch()
        n = feats.shape[0]
        lt = torch.zeros(n, dtype=torch.int32, device=self.device)
        y = torch.zeros(n, dtype=torch.float32, device=self.device) if want_y else None
        lo, hi = y_range if y_range is not None else (float("-inf"), float("inf"))
        agis_mlp_infer(self.ctx, params.data_ptr(), feats.data_ptr(), n, position_class, lt.data_ptr(),
                       y.data_ptr() if want_y else 0, base.data_ptr() if base is not None else 0, lo, hi)
        return (lt, y) if want_y else lt

    def weighted_steps(self, pattern, mode="switch"):
        plan = agis_compile_pattern(make_pattern(pattern.k, pattern.adj8()), params=make_params(mode=mode))
        return [i for i in range(pattern.k) if plan.decision[i] and plan.f1[i] > 0]

    def learned_tables(self, params, feats, pattern, base=None, rows=None):
        """Q16 pick table per weighted step (position class min(i, 3)); with
        base (from step_log_weights) the network's output corrects f_approx;
        with rows (the training rows) the output is clamped, per class, to
        the range of the training targets."""
        ranges = {}
        if rows is not None and rows["rows"]:
            cls = rows["cls"].cpu().numpy()
            tg = rows["target"].cpu().numpy()
            for c in np.unique(cls):
                ranges[int(c)] = (float(tg[cls == c].min()), float(tg[cls == c].max()))
        out = {}
        for i in self.weighted_steps(pattern, "learned"):
            c = min(i, 3)
            out[i] = self.mlp_infer(params, feats, c, base=None if base is None else base[i],
                                    y_range=ranges.get(c) if rows is not None else None)
        return out

    def release_scratch(self):
        """Gives back the sampler memory the context keeps between estimates
        (agis_release_scratch)."""
        agis_release_scratch(self.ctx)

    def close(self):
        if self.ctx:
            agis_destroy(self.ctx)
            self.ctx = None


def mlp_init(seed: int, target_mean: float = 0.0, zero_output: bool = False):
    """Initial parameters (Xavier-uniform weights, zero biases, output bias
    at the mean target), as a host float32 array in the library's layout.
    zero_output: output weights start at zero, so the untrained network is
    the constant target_mean (for residual tables: exactly f_approx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h, i = 64, 8

    def xavier(fan_out, fan_in):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))

    w3 = xavier(1, h).ravel()
    if zero_output:
        w3 = np.zeros_like(w3)
    parts = [xavier(h, i).ravel(), np.zeros(h), xavier(h, h).ravel(), np.zeros(h), w3,
             np.array([target_mean])]
    return np.concatenate(parts).astype(np.float32)
