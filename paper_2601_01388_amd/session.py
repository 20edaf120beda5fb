"""Convenience layer over the C names: owns torch device buffers for a CSR
graph and keeps the handles alive.  Still argument marshalling only; the
estimator runs in libagis.so."""

from __future__ import annotations

import ctypes

import numpy as np

from . import (AGIS_CSR_VALIDATE, LC_MIN_DEFAULT, RECORD_DTYPE, RECORD_BYTES, agis_build_proposal_tables,
               agis_autotune, agis_create, agis_destroy, agis_dump_samples, agis_estimate, agis_estimate_batch,
               agis_graph_destroy,
               agis_load_csr, agis_set_launch, agis_tables_destroy, agis_tables_export, make_params, make_pattern,
               lib)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the AGIS library needs a ROCm GPU; none is visible")
    return torch


class Graph:
    def __init__(self, sess, off: np.ndarray, nbr: np.ndarray, validate: bool = True):
        torch = _torch()
        self.sess = sess
        self.n = int(off.shape[0] - 1)
        self.nnz = int(nbr.shape[0])
        dev = sess.device
        self.d_off = torch.from_numpy(np.ascontiguousarray(off, dtype=np.uint64).view(np.int64)).to(dev)
        nb = np.ascontiguousarray(nbr, dtype=np.uint32).view(np.int32)
        self.d_nbr = torch.from_numpy(nb if nb.size else np.zeros(1, dtype=np.int32)).to(dev)
        self.handle = agis_load_csr(sess.ctx, self.d_off.data_ptr(), self.d_nbr.data_ptr(), self.n, self.nnz,
                                    AGIS_CSR_VALIDATE if validate else 0)

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

    def set_launch(self, use_graphs=True, blocks_per_cu=0, grab=0, variant=0):
        agis_set_launch(self.ctx, use_graphs, blocks_per_cu, grab, variant)

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

    def close(self):
        if self.ctx:
            agis_destroy(self.ctx)
            self.ctx = None
