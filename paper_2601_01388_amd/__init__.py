"""Python binding of libagis.so (the C-ABI in include/agis.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  The functions keep the C names (``agis_create``,
``agis_load_csr``, ...) and take plain integers for device pointers and
streams; PyTorch is used by callers only to own device memory and streams.

The binding refuses to work without the built library: there is no CPU
fallback.  Build it with ``python -m paper_2601_01388_amd.build``.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libagis.so")

MAX_K = 8

AGIS_OK = 0
AGIS_E_INVALID_ARG = -1
AGIS_E_INVALID_CSR = -2
AGIS_E_PATTERN = -3
AGIS_E_ORDER = -4
AGIS_E_OOM = -5
AGIS_E_HIP = -6
AGIS_E_NOT_CONVERGED = -7
AGIS_E_UNSUPPORTED = -8
AGIS_E_CANCELLED = -9

AGIS_MODE_UNIFORM = 0
AGIS_MODE_SWITCH = 1
AGIS_MODE_ALWAYS = 2
AGIS_MODE_LEARNED = 3
MODE_BY_NAME = {"uniform": 0, "switch": 1, "always": 2, "learned": 3}

AGIS_CSR_VALIDATE = 1
AGIS_RUN_ROWTAB_AUTO = 0
AGIS_RUN_ROWTAB_ON = 1
AGIS_RUN_ROWTAB_OFF = 2
ROWTAB_BY_NAME = {"auto": 0, "on": 1, "off": 2}
AGIS_RUN_STEP1_BLOCKS = 4
AGIS_RUN_STEP1_FULL = 8
AGIS_RUN_HOST_ROUNDS = 16
AGIS_RUN_WAVE_SAMPLES = 32
STEP1_BY_NAME = {"auto": 0, "blocks": AGIS_RUN_STEP1_BLOCKS, "full": AGIS_RUN_STEP1_FULL}
AGIS_TERMS_ALL = 0
AGIS_TERMS_F1 = 1
AGIS_TERMS_F1_I1 = 2
TERMS_BY_NAME = {"all": 0, "f1": 1, "f1_i1": 2}
LC_MIN_DEFAULT = -10 * 65536

_ERRNAMES = {
    -1: "AGIS_E_INVALID_ARG", -2: "AGIS_E_INVALID_CSR", -3: "AGIS_E_PATTERN", -4: "AGIS_E_ORDER",
    -5: "AGIS_E_OOM", -6: "AGIS_E_HIP", -7: "AGIS_E_NOT_CONVERGED", -8: "AGIS_E_UNSUPPORTED",
    -9: "AGIS_E_CANCELLED",
}


class AgisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class agis_pattern(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("adj", ctypes.c_uint8 * MAX_K)]


class agis_plan(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32), ("aut", ctypes.c_uint32),
        ("order", ctypes.c_uint8 * MAX_K), ("bmask", ctypes.c_uint8 * MAX_K), ("b", ctypes.c_uint8 * MAX_K),
        ("f1", ctypes.c_uint8 * MAX_K), ("i1", ctypes.c_uint8 * MAX_K), ("ie", ctypes.c_uint8 * MAX_K),
        ("f2", ctypes.c_uint8 * MAX_K), ("decision", ctypes.c_uint8 * MAX_K),
        ("cert_num", ctypes.c_int32 * MAX_K), ("cert_den", ctypes.c_int32 * MAX_K),
    ]


class agis_run_params(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("beta_num", ctypes.c_int32), ("beta_den", ctypes.c_int32),
        ("pattern_id", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("terms", ctypes.c_uint32),
        ("eps", ctypes.c_double), ("delta", ctypes.c_double),
        ("check_every", ctypes.c_uint64), ("min_samples", ctypes.c_uint64),
        ("learned", ctypes.c_void_p * MAX_K),
        ("first_sample", ctypes.c_uint64),
        ("cancel", ctypes.c_void_p),
        ("batch_learned", ctypes.c_void_p),
    ]


class agis_tuning(ctypes.Structure):
    _fields_ = [("use_graphs", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("grab", ctypes.c_uint32),
                ("variant", ctypes.c_int32), ("seconds", ctypes.c_double), ("default_seconds", ctypes.c_double),
                ("hub_window", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class agis_result(ctypes.Structure):
    _fields_ = [
        ("estimate", ctypes.c_double), ("copies", ctypes.c_double), ("variance", ctypes.c_double),
        ("eps_hat", ctypes.c_double), ("n", ctypes.c_uint64), ("n_nonzero", ctypes.c_uint64),
        ("aut", ctypes.c_uint32), ("converged", ctypes.c_int32), ("seconds", ctypes.c_double),
        ("tables_seconds", ctypes.c_double), ("sample_kernel_seconds", ctypes.c_double),
        ("sample_launches", ctypes.c_uint64), ("plan", agis_plan),
    ]


RECORD_DTYPE = np.dtype([
    ("v", np.uint32, (MAX_K,)), ("num", np.uint64, (MAX_K,)), ("den", np.uint64, (MAX_K,)),
    ("x", np.float64), ("steps", np.int32), ("fail_step", np.int32),
])
RECORD_BYTES = RECORD_DTYPE.itemsize  # 176

# (name, restype, argtypes) of every symbol include/agis.h declares
_P = ctypes.c_void_p
_SIGNATURES = [
    ("agis_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, _P]),
    ("agis_destroy", None, [_P]),
    ("agis_last_error", ctypes.c_char_p, [_P]),
    ("agis_release_scratch", ctypes.c_int, [_P]),
    ("agis_load_csr", ctypes.c_int, [_P, _P, _P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_void_p)]),
    ("agis_graph_destroy", None, [_P]),
    ("agis_orient", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_void_p)]),
    ("agis_graph_export", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    ("agis_build_proposal_tables", ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_void_p)]),
    ("agis_tables_destroy", None, [_P]),
    ("agis_tables_export", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    ("agis_compile_pattern", ctypes.c_int, [ctypes.POINTER(agis_pattern), _P, ctypes.POINTER(agis_run_params),
                                            ctypes.POINTER(agis_plan)]),
    ("agis_estimate", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(agis_pattern), _P, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.POINTER(agis_run_params), ctypes.POINTER(agis_result)]),
    ("agis_estimate_noalloc", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(agis_pattern), _P, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.POINTER(agis_run_params),
                                             ctypes.POINTER(agis_result)]),
    ("agis_dump_samples", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(agis_pattern), _P, ctypes.c_uint64,
                                         ctypes.POINTER(agis_run_params), _P, ctypes.c_uint64, _P]),
    ("agis_meter_samples", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(agis_pattern), _P, ctypes.c_uint64,
                                          ctypes.POINTER(agis_run_params), _P, ctypes.c_uint64, _P]),
    ("agis_gather_bench", ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    ("agis_estimate_batch", ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, _P, _P, ctypes.c_uint64,
                                           ctypes.POINTER(agis_run_params), _P]),
    ("agis_set_launch", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32,
                                       ctypes.c_uint32]),
    ("agis_autotune", ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, _P, ctypes.c_uint64,
                                     ctypes.POINTER(agis_run_params), ctypes.POINTER(agis_tuning)]),
    ("agis_mlp_param_count", ctypes.c_int, []),
    ("agis_features", ctypes.c_int, [_P, _P, _P]),
    ("agis_learn_targets", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(agis_pattern), _P, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.POINTER(agis_run_params), _P, _P]),
    ("agis_learn_rows", ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                       _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    ("agis_step_log_weights", ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                             _P]),
    ("agis_mlp_grad", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, ctypes.c_uint64, ctypes.c_float, _P, _P]),
    ("agis_mlp_train", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_float, ctypes.c_uint64, _P]),
    ("agis_mlp_infer", ctypes.c_int, [_P, _P, _P, ctypes.c_uint64, ctypes.c_uint32, _P, ctypes.c_float,
                                      ctypes.c_float, _P, _P]),
    ("agis_concentrations", ctypes.c_int, [ctypes.c_uint32, _P, _P, _P, _P, _P]),
    ("agis_connected_patterns", ctypes.c_int, [ctypes.c_uint32, _P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    ("agis_step1_weights", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(agis_pattern), _P,
                                          ctypes.POINTER(agis_run_params), _P, ctypes.POINTER(ctypes.c_uint64)]),
    ("agis_fixed_point_tables", ctypes.c_int, [_P, _P]),
    ("agis_philox4x32_10", ctypes.c_int, [_P, _P, _P]),
]
EXPORTED = [s[0] for s in _SIGNATURES]

_lib = None


def lib():
    """Loads libagis.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_01388_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, rc: int, allow=()):
    if rc != AGIS_OK and rc not in allow:
        msg = lib().agis_last_error(ctx).decode() if ctx else ""
        raise AgisError(rc, msg)
    return rc


# ---------------------------------------------------------------- C names

def agis_create(device: int = 0, stream: int = 0):
    h = ctypes.c_void_p()
    _check(None, lib().agis_create(ctypes.byref(h), device, stream))
    return h


def agis_destroy(ctx):
    lib().agis_destroy(ctx)


def agis_last_error(ctx) -> str:
    return lib().agis_last_error(ctx).decode()


def agis_release_scratch(ctx):
    _check(ctx, lib().agis_release_scratch(ctx))


def agis_load_csr(ctx, off_ptr: int, nbr_ptr: int, n: int, nnz: int, flags: int = AGIS_CSR_VALIDATE):
    h = ctypes.c_void_p()
    _check(ctx, lib().agis_load_csr(ctx, off_ptr, nbr_ptr, n, nnz, flags, ctypes.byref(h)))
    return h


def agis_graph_destroy(g):
    lib().agis_graph_destroy(g)


def agis_build_proposal_tables(ctx, g, cv_seed: int = 0, lc_min_q16: int = LC_MIN_DEFAULT, exact_cv: bool = False):
    h = ctypes.c_void_p()
    _check(ctx, lib().agis_build_proposal_tables(ctx, g, cv_seed, lc_min_q16, 1 if exact_cv else 0, ctypes.byref(h)))
    return h


def agis_tables_destroy(t):
    lib().agis_tables_destroy(t)


def agis_tables_export(ctx, t, deg=0, s2=0, hits=0, trials=0, la=0, lc=0):
    _check(ctx, lib().agis_tables_export(ctx, t, deg or None, s2 or None, hits or None, trials or None, la or None,
                                         lc or None))


def make_pattern(k: int, adj) -> agis_pattern:
    p = agis_pattern()
    p.k = k
    for i, a in enumerate(adj):
        p.adj[i] = a
    return p


def make_params(mode="switch", beta=(4, 5), pattern_id=0, eps=0.0, delta=0.05, check_every=0, min_samples=0,
                learned=None, rowtab="auto", terms="all", first_sample=0, cancel=None,
                batch_learned=None, step1="auto", host_rounds=False, wave_samples=False) -> agis_run_params:
    """Run parameters.  cancel: a ctypes.c_int32 the caller may set while the
    call runs (kept alive by the caller); batch_learned: a ctypes array of
    n_patterns * MAX_K table pointers (kept alive by the caller)."""
    pr = agis_run_params()
    pr.mode = MODE_BY_NAME[mode] if isinstance(mode, str) else int(mode)
    pr.flags = (ROWTAB_BY_NAME[rowtab] if isinstance(rowtab, str) else int(rowtab)) | STEP1_BY_NAME[step1]
    if host_rounds:
        pr.flags |= AGIS_RUN_HOST_ROUNDS
    if wave_samples:
        pr.flags |= AGIS_RUN_WAVE_SAMPLES
    pr.terms = TERMS_BY_NAME[terms] if isinstance(terms, str) else int(terms)
    pr.beta_num, pr.beta_den = beta
    pr.pattern_id = pattern_id
    pr.eps = eps
    pr.delta = delta
    pr.check_every = check_every
    pr.min_samples = min_samples
    if learned:
        for i, ptr in learned.items():
            pr.learned[i] = ptr
    pr.first_sample = first_sample
    if cancel is not None:
        pr.cancel = ctypes.addressof(cancel)
    if batch_learned is not None:
        pr.batch_learned = ctypes.addressof(batch_learned)
    return pr


def batch_learned_array(tables_per_pattern):
    """A host array of n_patterns * MAX_K device pointers for
    agis_run_params.batch_learned: tables_per_pattern[i] maps step -> ptr
    (or is None)."""
    n = len(tables_per_pattern)
    arr = (ctypes.c_void_p * (n * MAX_K))()
    for i, tabs in enumerate(tables_per_pattern):
        for j, ptr in (tabs or {}).items():
            arr[i * MAX_K + j] = ptr
    return arr


def _order_arg(order):
    if order is None:
        return None, None
    buf = (ctypes.c_uint8 * MAX_K)(*list(order))
    return buf, ctypes.cast(buf, ctypes.c_void_p)


def agis_compile_pattern(pattern: agis_pattern, order=None, params: agis_run_params = None) -> agis_plan:
    out = agis_plan()
    keep, ptr = _order_arg(order)
    rc = lib().agis_compile_pattern(ctypes.byref(pattern), ptr, ctypes.byref(params) if params else None,
                                    ctypes.byref(out))
    if rc != AGIS_OK:
        raise AgisError(rc, "pattern compile failed")
    del keep
    return out


def agis_estimate(ctx, g, t, pattern: agis_pattern, n_samples: int, seed: int, params: agis_run_params,
                  order=None) -> agis_result:
    """The result carries .status: AGIS_OK, AGIS_E_NOT_CONVERGED or
    AGIS_E_CANCELLED (other codes raise)."""
    out = agis_result()
    keep, ptr = _order_arg(order)
    out.status = _check(ctx, lib().agis_estimate(ctx, g, t, ctypes.byref(pattern), ptr, n_samples, seed,
                                                 ctypes.byref(params), ctypes.byref(out)),
                        allow=(AGIS_E_NOT_CONVERGED, AGIS_E_CANCELLED))
    del keep
    return out


def agis_estimate_noalloc(ctx, g, t, pattern: agis_pattern, n_samples: int, seed: int, params: agis_run_params,
                          order=None) -> agis_result:
    """agis_estimate without device allocation (the library's fixed
    workspace); the result carries .status as agis_estimate's does."""
    out = agis_result()
    keep, ptr = _order_arg(order)
    out.status = _check(ctx, lib().agis_estimate_noalloc(ctx, g, t, ctypes.byref(pattern), ptr, n_samples, seed,
                                                         ctypes.byref(params), ctypes.byref(out)),
                        allow=(AGIS_E_NOT_CONVERGED, AGIS_E_CANCELLED))
    del keep
    return out


def agis_dump_samples(ctx, g, t, pattern: agis_pattern, seed: int, params: agis_run_params, idx_ptr: int, m: int,
                      out_ptr: int, order=None):
    keep, ptr = _order_arg(order)
    _check(ctx, lib().agis_dump_samples(ctx, g, t, ctypes.byref(pattern), ptr, seed, ctypes.byref(params), idx_ptr,
                                        m, out_ptr))
    del keep


def agis_meter_samples(ctx, g, t, pattern: agis_pattern, seed: int, params: agis_run_params, idx_ptr: int, m: int,
                       out_ptr: int, order=None):
    keep, ptr = _order_arg(order)
    _check(ctx, lib().agis_meter_samples(ctx, g, t, ctypes.byref(pattern), ptr, seed, ctypes.byref(params), idx_ptr,
                                         m, out_ptr))
    del keep


def agis_gather_bench(ctx, buf_ptr: int, nbytes: int, seg_bytes: int, dependent: bool, waves_per_cu: int,
                      rounds: int, seed: int, sink_ptr: int):
    """(seconds, useful_bytes) of one random-gather run."""
    sec = ctypes.c_double()
    ub = ctypes.c_double()
    _check(ctx, lib().agis_gather_bench(ctx, buf_ptr, nbytes, seg_bytes, 1 if dependent else 0, waves_per_cu, rounds,
                                        seed, sink_ptr, ctypes.byref(sec), ctypes.byref(ub)))
    return float(sec.value), float(ub.value)


def agis_estimate_batch(ctx, g, t, patterns, budgets, seed: int, params: agis_run_params):
    """patterns: list of agis_pattern; budgets: list of ints.  Returns a
    list of agis_result (NOT_CONVERGED is reported in each result)."""
    n = len(patterns)
    arr = (agis_pattern * n)(*patterns)
    bud = (ctypes.c_uint64 * n)(*budgets)
    out = (agis_result * n)()
    rc = _check(ctx, lib().agis_estimate_batch(ctx, g, t, n, ctypes.cast(arr, _P), ctypes.cast(bud, _P), seed,
                                               ctypes.byref(params), ctypes.cast(out, _P)),
                allow=(AGIS_E_NOT_CONVERGED, AGIS_E_CANCELLED))
    res = list(out)
    for r in res:
        r.status = rc
    return res


def agis_set_launch(ctx, use_graphs: bool = True, blocks_per_cu: int = 0, grab: int = 0, variant: int = 0,
                    hub_window: int = 0):
    _check(ctx, lib().agis_set_launch(ctx, 1 if use_graphs else 0, blocks_per_cu, grab, variant, hub_window))


def agis_autotune(ctx, g, t, patterns, pilot_samples: int, params: agis_run_params) -> agis_tuning:
    n = len(patterns)
    arr = (agis_pattern * n)(*patterns)
    out = agis_tuning()
    _check(ctx, lib().agis_autotune(ctx, g, t, n, ctypes.cast(arr, _P), pilot_samples, ctypes.byref(params),
                                    ctypes.byref(out)))
    return out


def agis_mlp_param_count() -> int:
    return int(lib().agis_mlp_param_count())


def agis_features(ctx, t, feats_ptr: int):
    _check(ctx, lib().agis_features(ctx, t, feats_ptr))


def agis_learn_targets(ctx, g, t, pattern: agis_pattern, n_samples: int, seed: int, params: agis_run_params,
                       sums_ptr: int, counts_ptr: int, order=None):
    keep, ptr = _order_arg(order)
    _check(ctx, lib().agis_learn_targets(ctx, g, t, ctypes.byref(pattern), ptr, n_samples, seed, ctypes.byref(params),
                                         sums_ptr, counts_ptr))
    del keep


def agis_learn_rows(ctx, sums_ptr, counts_ptr, k, n, step_mask, min_count, vtx_ptr, cls_ptr, target_ptr,
                    weight_ptr, base_ptr=0) -> int:
    rows = ctypes.c_uint64()
    _check(ctx, lib().agis_learn_rows(ctx, sums_ptr, counts_ptr, k, n, step_mask, min_count, base_ptr or None,
                                      vtx_ptr, cls_ptr, target_ptr, weight_ptr, ctypes.byref(rows)))
    return int(rows.value)


def agis_step_log_weights(ctx, t, b, f1, ie, f2, out_ptr):
    _check(ctx, lib().agis_step_log_weights(ctx, t, b, f1, ie, f2, out_ptr))


def agis_mlp_grad(ctx, params_ptr, feats_ptr, vtx_ptr, cls_ptr, target_ptr, weight_ptr, rows, weight_sum, grad_ptr,
                  loss_ptr=0):
    _check(ctx, lib().agis_mlp_grad(ctx, params_ptr, feats_ptr, vtx_ptr, cls_ptr, target_ptr, weight_ptr, rows,
                                    weight_sum, grad_ptr, loss_ptr or None))


def agis_mlp_train(ctx, params_ptr, feats_ptr, vtx_ptr, cls_ptr, target_ptr, weight_ptr, rows, epochs, batch, lr,
                   shuffle_seed):
    losses = (ctypes.c_float * max(epochs, 1))()
    _check(ctx, lib().agis_mlp_train(ctx, params_ptr, feats_ptr, vtx_ptr, cls_ptr, target_ptr, weight_ptr, rows,
                                     epochs, batch, lr, shuffle_seed, ctypes.cast(losses, _P)))
    return [float(x) for x in losses[:epochs]]


def agis_mlp_infer(ctx, params_ptr, feats_ptr, n, position_class, lt_ptr, y_ptr=0, base_ptr=0,
                   y_min=float("-inf"), y_max=float("inf")):
    _check(ctx, lib().agis_mlp_infer(ctx, params_ptr, feats_ptr, n, position_class, base_ptr or None, y_min, y_max,
                                     lt_ptr, y_ptr or None))


def agis_step1_weights(ctx, g, t, pattern: agis_pattern, params: agis_run_params, q1_ptr, order=None) -> int:
    buf, optr = _order_arg(order)
    total = ctypes.c_uint64()
    _check(ctx, lib().agis_step1_weights(ctx, g, t, ctypes.byref(pattern), optr, ctypes.byref(params), q1_ptr,
                                         ctypes.byref(total)))
    return int(total.value)


def agis_orient(ctx, g):
    h = ctypes.c_void_p()
    _check(ctx, lib().agis_orient(ctx, g, ctypes.byref(h)))
    return h.value


def agis_graph_export(ctx, g):
    """(n, nnz, off_ptr, nbr_ptr) of a graph (device pointers)."""
    n = ctypes.c_uint64()
    nnz = ctypes.c_uint64()
    off = ctypes.c_void_p()
    nbr = ctypes.c_void_p()
    _check(ctx, lib().agis_graph_export(ctx, g, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(off),
                                        ctypes.byref(nbr)))
    return int(n.value), int(nnz.value), off.value, nbr.value


def agis_connected_patterns(k: int) -> list:
    """Every connected k-vertex pattern up to isomorphism, as agis_pattern."""
    cnt = ctypes.c_uint32()
    _check(None, lib().agis_connected_patterns(k, None, 0, ctypes.byref(cnt)))
    arr = (agis_pattern * max(cnt.value, 1))()
    _check(None, lib().agis_connected_patterns(k, ctypes.cast(arr, _P), cnt.value, ctypes.byref(cnt)))
    return [arr[i] for i in range(cnt.value)]


def agis_concentrations(patterns, copies):
    """(conc_edge, induced, conc_induced) as numpy arrays."""
    n = len(patterns)
    arr = (agis_pattern * n)(*patterns)
    c = np.ascontiguousarray(copies, dtype=np.float64)
    ce = np.zeros(n)
    ind = np.zeros(n)
    ci = np.zeros(n)
    _check(None, lib().agis_concentrations(n, ctypes.cast(arr, _P), c.ctypes.data, ce.ctypes.data, ind.ctypes.data,
                                           ci.ctypes.data))
    return ce, ind, ci


def agis_fixed_point_tables():
    lt = np.zeros(4096, dtype=np.int32)
    et = np.zeros(4096, dtype=np.uint32)
    _check(None, lib().agis_fixed_point_tables(lt.ctypes.data, et.ctypes.data))
    return lt, et


def agis_philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _check(None, lib().agis_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data))
    return [int(x) for x in o]
