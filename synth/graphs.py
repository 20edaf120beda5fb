"""Seeded synthetic data graphs in symmetric CSR form.

Layout (the one every consumer expects):
  * ``off``: uint64[n + 1], row offsets, ``off[0] == 0``, ``off[n] == nnz``;
  * ``nbr``: uint32[nnz], neighbour ids, each row strictly ascending;
  * undirected: ``x`` in row ``v`` iff ``v`` in row ``x``; no self-loops;
    so ``nnz`` is twice the number of undirected edges.

Generators use numpy's PCG64 stream with an explicit seed; they are input
generators only and draw nothing on behalf of the estimator.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class CSR:
    off: np.ndarray  # uint64[n+1]
    nbr: np.ndarray  # uint32[nnz]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.nbr.shape[0])

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.off).astype(np.int64)

    def row(self, v: int) -> np.ndarray:
        return self.nbr[int(self.off[v]):int(self.off[v + 1])]

    def adjacency_sets(self) -> list:
        return [set(int(x) for x in self.row(v)) for v in range(self.n)]


def csr_from_edges(n: int, u, v, name: str = "") -> CSR:
    """Symmetrise, drop self-loops and duplicates, and sort an edge list."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if n > 0 and u.size:
        if u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n:
            raise ValueError("edge endpoint out of range")
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * np.int64(n) + dst)
    rows = key // n
    cols = (key % n).astype(np.uint32)
    counts = np.bincount(rows, minlength=n).astype(np.uint64)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=off[1:])
    return CSR(off=off, nbr=cols, name=name)


def chung_lu(n: int = 10_000, m: int = 100_000, gamma: float = 2.1, seed: int = 1) -> CSR:
    """Chung-Lu power-law graph with exactly ``m`` distinct undirected edges.

    Vertex ``i`` has weight ``(i + 1) ** (-1 / (gamma - 1))``; both endpoints
    of a candidate edge are drawn independently with probability
    proportional to weight, self-loops are discarded, and candidates are
    taken in draw order until ``m`` distinct edges exist.
    """
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds the number of vertex pairs")
    rng = np.random.Generator(np.random.PCG64(seed))
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    order_keys = np.empty(0, dtype=np.int64)
    batch = max(2 * m, 1024)
    while True:
        a = np.searchsorted(cdf, rng.random(batch), side="right").astype(np.int64)
        b = np.searchsorted(cdf, rng.random(batch), side="right").astype(np.int64)
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        keep = a != b
        lo = np.minimum(a[keep], b[keep])
        hi = np.maximum(a[keep], b[keep])
        order_keys = np.concatenate([order_keys, lo * n + hi])
        uniq, first = np.unique(order_keys, return_index=True)
        if uniq.size >= m:
            chosen = uniq[np.argsort(first, kind="stable")[:m]]
            break
    return csr_from_edges(n, chosen // n, chosen % n, name=f"chung_lu_n{n}_m{m}_g{gamma}_s{seed}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 20, chunk: int = 1 << 24) -> CSR:
    """R-MAT graph: ``edge_factor * 2**scale`` recursive-quadrant draws.

    Each draw descends ``scale`` levels; at each level the quadrant is
    (0,0) w.p. a, (0,1) w.p. b, (1,0) w.p. c, (1,1) otherwise.  No noise and
    no vertex permutation.  The result is symmetrised and deduplicated with
    self-loops removed.
    """
    n = 1 << scale
    total = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    ab, abc = a + b, a + b + c
    keys = []
    done = 0
    while done < total:
        cnt = min(chunk, total - done)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(cnt)
            bu = (r >= ab).astype(np.int64)
            bv = (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64)
            u = (u << 1) | bu
            v = (v << 1) | bv
        keep = u != v
        u, v = u[keep], v[keep]
        keys.append(np.unique(np.concatenate([u * n + v, v * n + u])))
        done += cnt
    key = np.unique(np.concatenate(keys)) if len(keys) > 1 else keys[0]
    rows = key // n
    cols = (key % n).astype(np.uint32)
    counts = np.bincount(rows, minlength=n).astype(np.uint64)
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=off[1:])
    return CSR(off=off, nbr=cols, name=f"rmat{scale}_ef{edge_factor}_s{seed}")


def rmat_device(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                seed: int = 24, device: str = "cuda"):
    """The same R-MAT recipe as ``rmat``, drawn on a GPU with torch's
    counter-based generator (a different stream from ``rmat``'s, so a
    different graph for the same seed): for scales whose host generation
    takes minutes.  Returns (off int64[n+1], nbr int32[nnz]) device tensors
    of the symmetrised, deduplicated, loop-free CSR (off holds uint64
    values, nbr uint32 ids)."""
    import torch
    n = 1 << scale
    total = edge_factor * n
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    ab, abc = a + b, a + b + c
    keys = []
    chunk = 1 << 26
    done = 0
    while done < total:
        cnt = min(chunk, total - done)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for _ in range(scale):
            r = torch.rand(cnt, generator=gen, device=device, dtype=torch.float64)
            u = (u << 1) | (r >= ab).to(torch.int64)
            v = (v << 1) | (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64)
            del r
        keep = u != v
        u, v = u[keep], v[keep]
        keys.append(torch.unique(torch.cat([u * n + v, v * n + u])))
        del u, v, keep
        done += cnt
    key = torch.unique(torch.cat(keys)) if len(keys) > 1 else keys[0]
    del keys
    rows = torch.div(key, n, rounding_mode="floor")
    nbr = (key - rows * n).to(torch.int32)
    counts = torch.bincount(rows, minlength=n)
    del key, rows
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(counts, 0)
    return off, nbr


def tiny_graph(n: int, p: float, seed: int) -> CSR:
    """Erdos-Renyi G(n, p) for brute-force checks on a handful of vertices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    us, vs = [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p:
                us.append(i)
                vs.append(j)
    return csr_from_edges(n, us, vs, name=f"gnp_{n}_{p}_{seed}")


def skewed_tiny_graph(n: int, seed: int, hubs: int = 2, p_hub: float = 0.8, p: float = 0.2) -> CSR:
    """Small graph with a few hub vertices, for tests that need degree skew."""
    rng = np.random.Generator(np.random.PCG64(seed))
    us, vs = [], []
    for i in range(n):
        for j in range(i + 1, n):
            q = p_hub if (i < hubs or j < hubs) else p
            if rng.random() < q:
                us.append(i)
                vs.append(j)
    return csr_from_edges(n, us, vs, name=f"skew_{n}_{seed}")


def complete_graph(n: int) -> CSR:
    us, vs = np.triu_indices(n, 1)
    return csr_from_edges(n, us, vs, name=f"K{n}")


def ring_graph(n: int) -> CSR:
    us = np.arange(n)
    return csr_from_edges(n, us, (us + 1) % n, name=f"C{n}")


def star_graph(leaves: int) -> CSR:
    return csr_from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1), name=f"K1_{leaves}")


def complete_bipartite(a: int, b: int) -> CSR:
    us = np.repeat(np.arange(a), b)
    vs = np.tile(np.arange(a, a + b), a)
    return csr_from_edges(a + b, us, vs, name=f"K{a}_{b}")


# ---------------------------------------------------------------- counter-based R-MAT

_GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix_draws(seed: int, counters: np.ndarray) -> np.ndarray:
    """Draws `counters` of the counter-based SplitMix64 stream of `seed`
    (Steele, Lea and Flood, OOPSLA 2014): mix(seed + (i + 1) * gamma)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def rmat_counter_edges(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                       seed: int = 30, first: int = 0, count: int = None):
    """Endpoints (u, v) of edges [first, first + count) of the counter-based
    R-MAT stream that the GPU generator (synth/csrc/rmat_gen.hip) draws:
    level l of edge e uses draw e * 32 + l, top 53 bits over 2^53."""
    total = edge_factor << scale
    count = total - first if count is None else count
    e = np.arange(first, first + count, dtype=np.uint64)
    u = np.zeros(count, dtype=np.uint64)
    v = np.zeros(count, dtype=np.uint64)
    ab, abc = a + b, a + b + c
    for lvl in range(scale):
        r = (splitmix_draws(seed, e * np.uint64(32) + np.uint64(lvl)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        u = (u << np.uint64(1)) | (r >= ab).astype(np.uint64)
        v = (v << np.uint64(1)) | (((r >= a) & (r < ab)) | (r >= abc)).astype(np.uint64)
    return u.astype(np.int64), v.astype(np.int64)


def rmat_counter(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                 seed: int = 30) -> CSR:
    """Host generation of the counter-based R-MAT graph (small scales): the
    graph rmat_gpu builds for the same arguments."""
    u, v = rmat_counter_edges(scale, edge_factor, a, b, c, seed)
    return csr_from_edges(1 << scale, u, v, name=f"rmatc{scale}_ef{edge_factor}_s{seed}")


_GENLIB = None


def _genlib():
    import ctypes
    import os
    global _GENLIB
    if _GENLIB is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynthgen.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(path)
        P, u64, u32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        L.synth_rmat_count.argtypes = [P, u64, u32, dbl, dbl, dbl, u64, P]
        L.synth_rmat_fill.argtypes = [P, P, P, u64, u32, dbl, dbl, dbl, u64, P]
        L.synth_sort_dedup_rows.argtypes = [P, P, u64, P, P, u64, P]
        L.synth_compact_rows.argtypes = [P, P, P, u64, P, u64, P]
        for f in (L.synth_rmat_count, L.synth_rmat_fill, L.synth_sort_dedup_rows, L.synth_compact_rows):
            f.restype = ctypes.c_int
        _GENLIB = L
    return _GENLIB


def rmat_gpu(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
             seed: int = 30, device: str = "cuda", stage_bytes: int = 8 << 30):
    """The counter-based R-MAT graph built on the GPU in place (count the
    degrees, scatter both directions into rows, sort and deduplicate each
    row, move the rows onto the deduplicated offsets): the peak is the
    undeduplicated neighbour array plus two offset arrays, a degree array
    and the staging buffer.  Returns (off int64[n + 1], nbr int32[nnz])
    device tensors (off holds uint64 values, nbr uint32 ids); nbr is a view
    of the first nnz entries of the undeduplicated buffer."""
    import torch
    L = _genlib()
    n = 1 << scale
    total = edge_factor * n
    stream = torch.cuda.current_stream(torch.device(device)).cuda_stream

    def ok(rc, what):
        if rc != 0:
            raise RuntimeError(f"R-MAT generator: {what} failed ({rc})")

    deg = torch.zeros(n, dtype=torch.int32, device=device)
    ok(L.synth_rmat_count(deg.data_ptr(), total, scale, a, b, c, seed, stream), "count")
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(deg, 0, dtype=torch.int64, out=off[1:])
    slots = int(off[-1].item())
    nbr = torch.empty(max(slots, 1), dtype=torch.int32, device=device)
    deg.zero_()
    ok(L.synth_rmat_fill(off.data_ptr(), deg.data_ptr(), nbr.data_ptr(), total, scale, a, b, c, seed, stream),
       "fill")
    stage = torch.empty(int(stage_bytes), dtype=torch.uint8, device=device)
    ok(L.synth_sort_dedup_rows(off.data_ptr(), nbr.data_ptr(), n, deg.data_ptr(), stage.data_ptr(), stage_bytes,
                               stream), "sort and deduplicate")
    new_off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(deg, 0, dtype=torch.int64, out=new_off[1:])
    del deg
    ok(L.synth_compact_rows(off.data_ptr(), new_off.data_ptr(), nbr.data_ptr(), n, stage.data_ptr(), stage_bytes,
                            stream), "compact")
    del stage, off
    nnz = int(new_off[-1].item())
    return new_off, nbr[:nnz]


def build_generator() -> str:
    """Compiles synth/csrc/rmat_gen.hip into synth/libsynthgen.so (gfx950)."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    out = os.path.join(here, "libsynthgen.so")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    arch = os.environ.get("AGIS_OFFLOAD_ARCH", "gfx950")
    cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={arch}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           os.path.join(here, "csrc", "rmat_gen.hip"), "-o", out + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed building libsynthgen.so:\n" + res.stdout + res.stderr)
    os.replace(out + ".tmp", out)
    return out
