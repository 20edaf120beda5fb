"""CPU oracle for the AGIS sampling estimator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it.

Pieces:
  * ``agis_oracle.c`` (built into ``liboracle.so`` with gcc): Philox,
    Lemire draws, Q16 log2 encoding, proposal tables, Algorithm 3 sampler,
    step distributions, exact counting judges;
  * ``pattern.py``: the pattern compiler (Algorithm 2, auxiliary arrays,
    decision function);
  * ``estimator.py``: Algorithm 1 statistics and the run-to-epsilon loop;
  * ``tree.py``: exact expectation over the whole sampling tree;
  * ``judges.py``: exact counts (brute force and closed forms).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .pattern import compile_pattern, matching_order, automorphisms, step_analysis  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "agis_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MAXK = 8
CERTAIN_ZERO = -(1 << 31)
LC_MIN_DEFAULT = -10 * 65536  # log2(2^-10) in Q16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Plan(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32),
        ("pattern_id", ctypes.c_uint32),
        ("bmask", ctypes.c_uint8 * MAXK),
        ("f1", ctypes.c_uint8 * MAXK),
        ("ie", ctypes.c_uint8 * MAXK),
        ("f2", ctypes.c_uint8 * MAXK),
        ("decision", ctypes.c_uint8 * MAXK),
        ("oriented", ctypes.c_uint8),
    ]


class Record(ctypes.Structure):
    _fields_ = [
        ("v", ctypes.c_uint32 * MAXK),
        ("num", ctypes.c_uint64 * MAXK),
        ("den", ctypes.c_uint64 * MAXK),
        ("x", ctypes.c_double),
        ("steps", ctypes.c_int32),
        ("fail_step", ctypes.c_int32),
    ]


RECORD_DTYPE = np.dtype([
    ("v", np.uint32, (MAXK,)),
    ("num", np.uint64, (MAXK,)),
    ("den", np.uint64, (MAXK,)),
    ("x", np.float64),
    ("steps", np.int32),
    ("fail_step", np.int32),
])
assert RECORD_DTYPE.itemsize == ctypes.sizeof(Record)


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("mean", ctypes.c_double), ("m2", ctypes.c_double),
                ("nonzero", ctypes.c_uint64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_bounded.argtypes = [P, u32, u32, u32, u32, u64]
        L.orc_bounded.restype = u64
        L.orc_log2fx.argtypes = [u64]
        L.orc_log2fx.restype = i32
        L.orc_weight_from_log.argtypes = [i32, i32]
        L.orc_weight_from_log.restype = u32
        L.orc_fixed_point_tables.argtypes = [P, P]
        L.orc_build_tables.argtypes = [P, P, u64, u32, u32, i32, ctypes.c_int, P, P, P, P, P, P]
        L.orc_build_tables_oriented.argtypes = [P, P, u64, P, P, u32, u32, i32, ctypes.c_int, P, P, P, P, P, P]
        L.orc_orient.argtypes = [P, P, u64, P, P]
        L.orc_orient.restype = u64
        L.orc_log_weights.argtypes = [P, P, ctypes.c_int, u64, P]
        L.orc_tables_at.argtypes = [P, P, P, u64, u32, u32, i32, ctypes.c_int, P, P, P, P, P, P]
        L.orc_step1_table.argtypes = [P, P, P, P, P, P]
        L.orc_step1_table.restype = u64
        L.orc_run.argtypes = [P, P, u64, u64, P, P, P, P, P, P, P, P, u64, u64, u64, u64, P, P, P]
        L.orc_run.restype = ctypes.c_int
        L.orc_run_indices.argtypes = [P, P, u64, u64, P, P, P, P, P, P, P, P, u64, u64, P, u64, P]
        L.orc_run_indices.restype = ctypes.c_int
        L.orc_step_distribution.argtypes = [P, P, u64, u64, P, P, P, P, P, P, P, ctypes.c_int, P, P, P]
        L.orc_step_distribution.restype = u64
        L.orc_step_distribution_literal.argtypes = [P, P, u64, u64, P, P, P, P, ctypes.c_int, P, P, P]
        L.orc_step_distribution_literal.restype = u64
        L.orc_literal_terms.argtypes = [u64, u32, u32, u32, u32, ctypes.c_double, u64, P, P, P]
        L.orc_count_embeddings.argtypes = [P, P, u64, u64, P, P, u32]
        L.orc_count_embeddings.restype = u64
        L.orc_count_cliques.argtypes = [P, P, u64, u64, u32]
        L.orc_rooted_counts.argtypes = [P, P, u64, u64, P, P, u32, P]
        L.orc_rooted_counts.restype = u64
        L.orc_count_cliques.restype = u64
        L.orc_build_tables_parallel.argtypes = [P, P, u64, u32, u32, i32, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        L.orc_build_tables_parallel.restype = ctypes.c_int
        L.orc_run_parallel.argtypes = [P, P, u64, u64, P, P, P, P, P, P, P, P, u64, u64, u64, u64, ctypes.c_int, P]
        L.orc_run_parallel.restype = ctypes.c_int
        L.orc_run_indices_parallel.argtypes = [P, P, u64, u64, P, P, P, P, P, P, P, P, u64, u64, P, u64, ctypes.c_int,
                                               P]
        L.orc_run_indices_parallel.restype = ctypes.c_int
        L.orc_count_cliques_parallel.argtypes = [P, P, u64, u64, u32, ctypes.c_int]
        L.orc_count_cliques_parallel.restype = u64
        _lib = L
    return _lib


def _p(a):
    """The array's address (None: a null pointer)."""
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- RNG

def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return [int(x) for x in out]


def bounded(seed: int, c0: int, c1: int, c2: int, tag: int, rng: int) -> int:
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
    return int(lib().orc_bounded(_p(key), c0, c1, c2, tag, rng))


def log2fx(x: int) -> int:
    return int(lib().orc_log2fx(x))


def weight_from_log(lmax: int, lw: int) -> int:
    return int(lib().orc_weight_from_log(lmax, lw))


def fixed_point_tables():
    lt = np.zeros(4096, dtype=np.int32)
    et = np.zeros(4096, dtype=np.uint32)
    lib().orc_fixed_point_tables(_p(lt), _p(et))
    return lt, et


# ---------------------------------------------------------------- tables

class Tables:
    """Per-vertex proposal tables of Sec. 4.4 (host arrays)."""

    def __init__(self, g, cv_seed: int = 0, lc_min: int = LC_MIN_DEFAULT, exact_cv: bool = False,
                 adjacency=None, threads: int = 1):
        """adjacency: for an oriented g, the undirected graph that decides
        whether two out-neighbours are adjacent (C_v over out-neighbours).
        threads != 1: the OpenMP flavour (0 = all host threads; same
        entries, per vertex)."""
        n = g.n
        self.n = n
        self.deg = np.zeros(n, dtype=np.uint32)
        self.s2 = np.zeros(n, dtype=np.uint64)
        self.hits = np.zeros(n, dtype=np.uint64)
        self.trials = np.zeros(n, dtype=np.uint64)
        self.la = np.zeros(n, dtype=np.int32)
        self.lc = np.zeros(n, dtype=np.int32)
        self.cv_seed = cv_seed
        self.lc_min = lc_min
        self.exact_cv = exact_cv
        off = np.ascontiguousarray(g.off, dtype=np.uint64)
        nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
        if adjacency is None and threads != 1:
            lib().orc_build_tables_parallel(_p(off), _p(nbr), n, cv_seed & 0xFFFFFFFF, cv_seed >> 32, lc_min,
                                            1 if exact_cv else 0, threads, _p(self.deg), _p(self.s2), _p(self.hits),
                                            _p(self.trials), _p(self.la), _p(self.lc))
        elif adjacency is None:
            lib().orc_build_tables(_p(off), _p(nbr), n, cv_seed & 0xFFFFFFFF, cv_seed >> 32, lc_min,
                                   1 if exact_cv else 0, _p(self.deg), _p(self.s2), _p(self.hits),
                                   _p(self.trials), _p(self.la), _p(self.lc))
        else:
            aoff = np.ascontiguousarray(adjacency.off, dtype=np.uint64)
            anbr = np.ascontiguousarray(adjacency.nbr, dtype=np.uint32)
            lib().orc_build_tables_oriented(_p(off), _p(nbr), n, _p(aoff), _p(anbr), cv_seed & 0xFFFFFFFF,
                                            cv_seed >> 32, lc_min, 1 if exact_cv else 0, _p(self.deg), _p(self.s2),
                                            _p(self.hits), _p(self.trials), _p(self.la), _p(self.lc))

    @classmethod
    def degrees_only(cls, g) -> "Tables":
        """The degrees alone, d(v) = off[v + 1] - off[v]; the other entries
        are unset and reach the sampler as null pointers.  Enough for plans
        that read no other entry -- every step uniform (f_uniform, Algorithm
        3 with D(i) = 0), or every weighted step without the T[I1] and T[F2]
        terms (a star: its centre weighted by T[F1] alone, its leaves
        trivial) -- on graphs whose full tables would take too long to build
        on the host."""
        t = cls.__new__(cls)
        t.n = g.n
        off = np.asarray(g.off, dtype=np.uint64)
        t.deg = np.empty(g.n, dtype=np.uint32)
        step = 1 << 26
        for lo in range(0, g.n, step):
            hi = min(g.n, lo + step)
            t.deg[lo:hi] = (off[lo + 1:hi + 1] - off[lo:hi]).astype(np.uint32)
        t.s2 = t.hits = t.trials = t.la = t.lc = None
        t.cv_seed = 0
        t.lc_min = LC_MIN_DEFAULT
        t.exact_cv = False
        return t

    def cv(self) -> np.ndarray:
        """Clustering coefficient hits / trials (0 where undefined)."""
        t = self.trials.astype(np.float64)
        return np.where(t > 0, self.hits.astype(np.float64) / np.maximum(t, 1), 0.0)


TERMS = ("all", "f1", "f1_i1")


def tables_at(g, vertices, cv_seed: int = 0, lc_min: int = LC_MIN_DEFAULT, exact_cv: bool = False) -> dict:
    """Table entries (deg, s2, hits, trials, la, lc) of the listed vertices
    only, by the same definitions as Tables."""
    vs = np.ascontiguousarray(vertices, dtype=np.uint64)
    m = vs.size
    out = {"deg": np.zeros(m, np.uint32), "s2": np.zeros(m, np.uint64), "hits": np.zeros(m, np.uint64),
           "trials": np.zeros(m, np.uint64), "la": np.zeros(m, np.int32), "lc": np.zeros(m, np.int32)}
    off = np.ascontiguousarray(g.off, dtype=np.uint64)
    nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
    lib().orc_tables_at(_p(off), _p(nbr), _p(vs), m, cv_seed & 0xFFFFFFFF, cv_seed >> 32, lc_min, int(exact_cv),
                        _p(out["deg"]), _p(out["s2"]), _p(out["hits"]), _p(out["trials"]), _p(out["la"]),
                        _p(out["lc"]))
    return out


def orient(g):
    """The degree orientation of a symmetric CSR: v -> w kept iff
    (d(v), v) < (d(w), w).  Returns a CSR of out-neighbour lists."""
    from synth.graphs import CSR
    off = np.ascontiguousarray(g.off, dtype=np.uint64)
    nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
    oo = np.zeros(g.n + 1, dtype=np.uint64)
    on = np.zeros(max(g.nnz // 2, 1), dtype=np.uint32)
    m = int(lib().orc_orient(_p(off), _p(nbr), g.n, _p(oo), _p(on)))
    return CSR(off=oo, nbr=on[:m].copy(), name=(g.name or "") + "_oriented")


def make_plan(compiled: dict, pattern_id: int = 0, terms: str = "all", oriented: bool = False) -> Plan:
    """terms: the factors of f_approx kept in the weights -- all three, or
    the incremental versions of the paper's analysis of the approximation
    (T[F1] only; T[F1] T[I1]).  Dropping T[I1] or T[F2] sets its exponent
    (ie or f2) to zero."""
    assert terms in TERMS
    P = Plan()
    P.k = compiled["k"]
    P.pattern_id = pattern_id
    for i, s in enumerate(compiled["steps"]):
        P.bmask[i] = s["bmask"]
        P.f1[i] = s["f1"]
        P.ie[i] = 0 if terms == "f1" else s["ie"]
        P.f2[i] = s["f2"] if terms == "all" else 0
        P.decision[i] = s["decision"]
    P.oriented = 1 if oriented else 0
    return P


class Sampler:
    """Algorithm 3 over one graph/pattern; all state on the host."""

    def __init__(self, g, tables: Tables, compiled: dict, seed: int, pattern_id: int = 0, learned=None,
                 terms: str = "all", oriented: bool = False):
        """oriented: g is the degree orientation of a graph (orient) and the
        pattern a clique; each clique is one trajectory, so the mean of X
        counts cliques (k! embeddings each)."""
        self.g = g
        self.off = np.ascontiguousarray(g.off, dtype=np.uint64)
        self.nbr = np.ascontiguousarray(g.nbr, dtype=np.uint32)
        self.t = tables
        self.compiled = compiled
        self.plan = make_plan(compiled, pattern_id, terms, oriented)
        self.seed = seed
        self._learned = learned
        if learned is not None:
            self._lt_arrays = [None if learned.get(i) is None else np.ascontiguousarray(learned[i], dtype=np.int32)
                               for i in range(MAXK)]
            self._lt_ptrs = (ctypes.c_void_p * MAXK)(*[None if a is None else a.ctypes.data for a in self._lt_arrays])
            self._lt = ctypes.cast(self._lt_ptrs, ctypes.c_void_p)
        else:
            self._lt = None
        self.q1 = np.zeros(g.n, dtype=np.uint32)
        self.pre1 = np.zeros(g.n, dtype=np.uint64)
        self.Q1 = 0
        weighted0 = compiled["steps"][0]["decision"] == 1 and compiled["steps"][0]["f1"] > 0
        if weighted0 and g.n > 0:
            lt0 = None
            if learned is not None and self._lt_arrays[0] is not None:
                lt0 = _p(self._lt_arrays[0])
            self.Q1 = int(lib().orc_step1_table(self._graph_struct(), self._tables_struct(), ctypes.byref(self.plan),
                                               lt0, _p(self.q1), _p(self.pre1)))

    def _graph_struct(self):
        class G(ctypes.Structure):
            _fields_ = [("n", ctypes.c_uint64), ("nnz", ctypes.c_uint64), ("off", ctypes.c_void_p),
                        ("nbr", ctypes.c_void_p)]
        self._gs = G(self.g.n, self.g.nnz, self.off.ctypes.data, self.nbr.ctypes.data)
        return ctypes.byref(self._gs)

    def _tables_struct(self):
        class T(ctypes.Structure):
            _fields_ = [("deg", ctypes.c_void_p), ("s2", ctypes.c_void_p), ("la", ctypes.c_void_p),
                        ("lc", ctypes.c_void_p)]
        t = self.t
        addr = [None if a is None else a.ctypes.data for a in (t.deg, t.s2, t.la, t.lc)]
        self._ts = T(*addr)
        return ctypes.byref(self._ts)

    def _common(self):
        t = self.t
        return (_p(self.off), _p(self.nbr), self.g.n, self.g.nnz, _p(t.deg), _p(t.s2), _p(t.la), _p(t.lc),
                ctypes.byref(self.plan), self._lt, _p(self.q1), _p(self.pre1), self.Q1, self.seed)

    def run(self, start: int, count: int, stats: Stats = None, want_x: bool = False, want_records: bool = False):
        st = stats if stats is not None else Stats()
        xs = np.zeros(count, dtype=np.float64) if want_x else None
        recs = np.zeros(count, dtype=RECORD_DTYPE) if want_records else None
        rc = lib().orc_run(*self._common(), start, count, ctypes.byref(st),
                           _p(xs) if xs is not None else None, _p(recs) if recs is not None else None)
        if rc != 0:
            raise MemoryError("oracle scratch allocation failed")
        return st, xs, recs

    def records(self, indices, threads: int = 1) -> np.ndarray:
        """threads != 1: the OpenMP flavour (0 = all host threads)."""
        idx = np.ascontiguousarray(indices, dtype=np.uint64)
        recs = np.zeros(idx.size, dtype=RECORD_DTYPE)
        if threads != 1:
            rc = lib().orc_run_indices_parallel(*self._common(), _p(idx), idx.size, threads, _p(recs))
            rc = 0 if rc > 0 else -1
        else:
            rc = lib().orc_run_indices(*self._common(), _p(idx), idx.size, _p(recs))
        if rc != 0:
            raise MemoryError("oracle scratch allocation failed")
        return recs

    def run_parallel(self, start: int, count: int, threads: int = 0):
        """Samples [start, start + count) on host threads, one sampler per
        thread over contiguous blocks merged in block order: (Stats, threads
        used)."""
        st = Stats()
        rc = lib().orc_run_parallel(*self._common(), start, count, threads, ctypes.byref(st))
        if rc < 0:
            raise MemoryError("oracle scratch allocation failed (or fewer threads than asked)")
        return st, rc

    def log_weights(self, i: int) -> np.ndarray:
        """f_approx Q16 log weight of every vertex at step i (certain zeros
        are INT32_MIN)."""
        out = np.zeros(max(self.g.n, 1), dtype=np.int32)
        lib().orc_log_weights(self._tables_struct(), ctypes.byref(self.plan), i, self.g.n, _p(out))
        return out[: self.g.n].copy()

    def step_distribution(self, i: int, tau):
        t = self.t
        n = self.g.n
        tau_a = np.zeros(MAXK, dtype=np.uint32)
        tau_a[:len(tau)] = tau
        out_v = np.zeros(max(n, 1), dtype=np.uint32)
        out_w = np.zeros(max(n, 1), dtype=np.uint64)
        m = lib().orc_step_distribution(_p(self.off), _p(self.nbr), n, self.g.nnz, _p(t.deg), _p(t.s2), _p(t.la),
                                        _p(t.lc), ctypes.byref(self.plan), self._lt, _p(self.q1), i, _p(tau_a),
                                        _p(out_v), _p(out_w))
        return out_v[:m].copy(), out_w[:m].copy()

    def step_distribution_literal(self, i: int, tau, cv: np.ndarray):
        t = self.t
        n = self.g.n
        tau_a = np.zeros(MAXK, dtype=np.uint32)
        tau_a[:len(tau)] = tau
        cvv = np.ascontiguousarray(cv, dtype=np.float64)
        out_v = np.zeros(max(n, 1), dtype=np.uint32)
        out_w = np.zeros(max(n, 1), dtype=np.float64)
        m = lib().orc_step_distribution_literal(_p(self.off), _p(self.nbr), n, self.g.nnz, _p(t.deg), _p(t.s2),
                                                _p(cvv), ctypes.byref(self.plan), i, _p(tau_a), _p(out_v),
                                                _p(out_w))
        return out_v[:m].copy(), out_w[:m].copy()


def literal_terms(d, b, f1, ie, f2, cv, s2):
    a = ctypes.c_double()
    c = ctypes.c_double()
    e = ctypes.c_double()
    lib().orc_literal_terms(d, b, f1, ie, f2, cv, s2, ctypes.byref(a), ctypes.byref(c), ctypes.byref(e))
    return a.value, c.value, e.value
