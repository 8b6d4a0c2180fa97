"""ctypes binding over libphg.so with the C ABI's names (argument marshalling only).

Every function takes numpy arrays (host inputs) or integer device pointers
(``phg_gradient_async``, ``phg_bind_workspace``, ``phg_bind_stream``) and
raises ``PhgError`` carrying the status code and the library's message when
a call does not return PHG_OK.  All computation happens in the library's HIP
kernels; there is no Python or CPU fallback: if libphg.so is missing the
import of this module's loader fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphg.so")

PHG_OK = 0
PHG_ERR_ARG = -1
PHG_ERR_STATE = -2
PHG_ERR_OOM = -3
PHG_ERR_DEVICE = -4
PHG_ERR_NUMERIC = -5
PHG_ERR_BUSY = -6
PHG_FP64 = 0
PHG_FP32_SCALED = 1
PHG_SCHEDULE_AUTO = 0
PHG_SCHEDULE_LEVELS = 1
PHG_SCHEDULE_BLOCKS = 2
PHG_SCHEDULE_QUEUE = 3

STATUS_NAMES = {0: "PHG_OK", -1: "PHG_ERR_ARG", -2: "PHG_ERR_STATE", -3: "PHG_ERR_OOM",
                -4: "PHG_ERR_DEVICE", -5: "PHG_ERR_NUMERIC", -6: "PHG_ERR_BUSY"}


class PhgError(RuntimeError):
    def __init__(self, status: int, message: str, where: str):
        self.status = status
        self.message = message
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_lib = None
_c = ctypes
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p

_SIGS = {
    "phg_create": [_c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.POINTER(_vp)],
    "phg_destroy": [_vp],
    "phg_last_error": [_vp],
    "phg_set_topology": [_vp, _ip],
    "phg_set_branch_lengths": [_vp, _dp],
    "phg_set_eigen": [_vp, _dp, _dp, _dp],
    "phg_set_root_frequencies": [_vp, _dp],
    "phg_set_categories": [_vp, _dp, _dp],
    "phg_set_tip_states": [_vp, _ip],
    "phg_set_tip_partials": [_vp, _c.c_int, _dp],
    "phg_set_pattern_weights": [_vp, _dp],
    "phg_prepare": [_vp],
    "phg_set_schedule": [_vp, _c.c_int],
    "phg_log_likelihood": [_vp, _dp],
    "phg_gradient": [_vp, _dp, _dp],
    "phg_workspace_size": [_c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.POINTER(_c.c_size_t)],
    "phg_kernel_family_of": [_c.c_int, _c.c_int, _c.c_int, _c.POINTER(_c.c_int)],
    "phg_bind_workspace": [_vp, _vp, _c.c_size_t],
    "phg_bind_stream": [_vp, _vp],
    "phg_gradient_async": [_vp, _vp, _vp],
    "phg_gradient_async_noalloc": [_vp, _vp, _vp],
    "phg_get_schedule": [_vp, _c.POINTER(_c.c_int)],
    "phg_set_category_eigen": [_vp, _dp, _dp, _dp],
    "phg_set_time_tree": [_vp, _dp, _dp],
    "phg_set_branch_sets": [_vp, _ip, _c.c_int],
    "phg_time_tree_gradient": [_vp, _dp, _dp, _dp, _dp],
    "phg_gradient_branch_sets": [_vp, _dp, _dp],
    "phg_schedule_info": [_vp, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)],
    "phg_server_create": [_c.c_int, _c.c_size_t, _c.c_int, _c.POINTER(_vp)],
    "phg_server_destroy": [_vp],
    "phg_server_last_error": [_vp],
    "phg_server_register_tree": [_vp, _vp, _c.POINTER(_c.c_uint64)],
    "phg_server_submit": [_vp, _c.c_uint64, _dp, _c.POINTER(_c.c_uint64)],
    "phg_server_poll": [_vp, _c.c_uint64, _dp, _dp, _c.POINTER(_c.c_int)],
    "phg_server_poll_timed": [_vp, _c.c_uint64, _dp, _dp, _c.POINTER(_c.c_int),
                              _c.POINTER(_c.c_uint64), _c.POINTER(_c.c_uint64)],
    "phg_server_wait": [_vp, _c.c_uint64, _dp, _dp],
    "phg_server_release_tree": [_vp, _c.c_uint64],
    "phg_server_stats": [_vp, _c.POINTER(_c.c_uint64)],
    "phg_server_busy": [_vp, _c.POINTER(_c.c_uint64), _c.POINTER(_c.c_uint64)],
    "phg_profile_enable": [_vp, _c.c_int],
    "phg_profile_read": [_vp, _dp, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)],
    "phg_set_fp32_guard": [_vp, _c.c_double],
    "phg_fp32_saturation": [_vp, _dp],
    "phg_last_precision": [_vp, _c.POINTER(_c.c_int)],
    "phg_set_graphs": [_vp, _c.c_int],
    "phg_set_table_budget": [_vp, _c.c_size_t],
    "phg_table_slots": [_vp, _c.POINTER(_c.c_int)],
    "phg_graph_stats": [_vp, _c.POINTER(_c.c_uint64), _c.POINTER(_c.c_uint64)],
    "phg_set_tuning": [_c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.c_int],
    "phg_get_tuning": [_c.c_int, _c.c_int, _c.c_int, _c.c_int, _c.POINTER(_c.c_int)],
}

PHG_PROF_CLASSES = 4
PROF_NAMES = ("pmat", "post", "pre_grad", "finalize")


def lib():
    """Load libphg.so (built in-tree by paper_2303_04390_amd.build).

    PyTorch wheels for ROCm bundle their own HIP and HSA runtimes under the
    same sonames as the system ones libphg.so links against.  torch is
    imported first so that libphg.so binds to the runtime already in the
    process: one HIP runtime, so torch streams and memory are valid handles
    for the library.  (Loading libphg.so first would map a second runtime.)
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2303_04390_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name.endswith("last_error") else ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, ctx, where: str):
    if status != PHG_OK:
        msg = lib().phg_last_error(ctx)
        raise PhgError(status, (msg or b"").decode(), where)


def _f64(a, n: Optional[int] = None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _i32(a, n: Optional[int] = None):
    a = np.ascontiguousarray(a, dtype=np.int32)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _p(a):
    return a.ctypes.data_as(_dp if a.dtype == np.float64 else _ip)


# ------------------------------------------------------------ C ABI, same names

def phg_create(n_tips, n_patterns, n_states, n_categories, prec, device=0):
    out = _vp()
    st = lib().phg_create(n_tips, n_patterns, n_states, n_categories, prec, device,
                          ctypes.byref(out))
    _check(st, None, "phg_create")
    return out


def phg_destroy(ctx):
    lib().phg_destroy(ctx)


def phg_last_error(ctx=None) -> str:
    return (lib().phg_last_error(ctx) or b"").decode()


def phg_set_topology(ctx, parent):
    a = _i32(parent)
    _check(lib().phg_set_topology(ctx, _p(a)), ctx, "phg_set_topology")


def phg_set_branch_lengths(ctx, b):
    a = _f64(b)
    _check(lib().phg_set_branch_lengths(ctx, _p(a)), ctx, "phg_set_branch_lengths")


def phg_set_eigen(ctx, V, Vinv, lam):
    a, b, c = _f64(V), _f64(Vinv), _f64(lam)
    _check(lib().phg_set_eigen(ctx, _p(a), _p(b), _p(c)), ctx, "phg_set_eigen")


def phg_set_category_eigen(ctx, V, Vinv, lam):
    a, b, c = _f64(V), _f64(Vinv), _f64(lam)
    _check(lib().phg_set_category_eigen(ctx, _p(a), _p(b), _p(c)), ctx, "phg_set_category_eigen")


def phg_set_root_frequencies(ctx, pi):
    a = _f64(pi)
    _check(lib().phg_set_root_frequencies(ctx, _p(a)), ctx, "phg_set_root_frequencies")


def phg_set_categories(ctx, rates, weights):
    a, b = _f64(rates), _f64(weights)
    _check(lib().phg_set_categories(ctx, _p(a), _p(b)), ctx, "phg_set_categories")


def phg_set_tip_states(ctx, codes):
    a = _i32(codes)
    _check(lib().phg_set_tip_states(ctx, _p(a)), ctx, "phg_set_tip_states")


def phg_set_tip_partials(ctx, tip: int, partials):
    """partials: [C, S] array (tip's general partial vector), or None to
    revert the tip to its code."""
    if partials is None:
        _check(lib().phg_set_tip_partials(ctx, int(tip), None), ctx, "phg_set_tip_partials")
        return
    a = _f64(partials)
    _check(lib().phg_set_tip_partials(ctx, int(tip), _p(a)), ctx, "phg_set_tip_partials")


def phg_set_pattern_weights(ctx, w):
    a = _f64(w)
    _check(lib().phg_set_pattern_weights(ctx, _p(a)), ctx, "phg_set_pattern_weights")


def phg_set_schedule(ctx, mode: int):
    _check(lib().phg_set_schedule(ctx, mode), ctx, "phg_set_schedule")


def phg_prepare(ctx):
    _check(lib().phg_prepare(ctx), ctx, "phg_prepare")


def phg_log_likelihood(ctx) -> float:
    v = ctypes.c_double()
    _check(lib().phg_log_likelihood(ctx, ctypes.byref(v)), ctx, "phg_log_likelihood")
    return v.value


def phg_gradient(ctx, n_branches: int, want_logl: bool = True):
    """Returns (logl, grad[n_branches])."""
    g = np.empty(n_branches, np.float64)
    v = ctypes.c_double()
    st = lib().phg_gradient(ctx, ctypes.byref(v) if want_logl else None, _p(g))
    _check(st, ctx, "phg_gradient")
    return v.value, g


def phg_workspace_size(n_tips, n_patterns, n_states, n_categories, prec) -> int:
    v = ctypes.c_size_t()
    st = lib().phg_workspace_size(n_tips, n_patterns, n_states, n_categories, prec, ctypes.byref(v))
    _check(st, None, "phg_workspace_size")
    return v.value


PHG_KERNELS_FOUR_STATE, PHG_KERNELS_SMALL_MFMA, PHG_KERNELS_VECTOR_ALU, PHG_KERNELS_MFMA = 0, 1, 2, 3
KERNEL_FAMILY_NAMES = ("four_state", "small_mfma", "valu", "mfma")


def phg_kernel_family_of(n_states, n_categories, prec) -> int:
    v = ctypes.c_int()
    st = lib().phg_kernel_family_of(n_states, n_categories, prec, ctypes.byref(v))
    _check(st, None, "phg_kernel_family_of")
    return v.value


def phg_bind_workspace(ctx, device_ptr: int, nbytes: int):
    _check(lib().phg_bind_workspace(ctx, _vp(device_ptr), nbytes), ctx, "phg_bind_workspace")


def phg_bind_stream(ctx, hip_stream: int):
    _check(lib().phg_bind_stream(ctx, _vp(hip_stream)), ctx, "phg_bind_stream")


def phg_gradient_async(ctx, d_logl: int, d_grad: int):
    _check(lib().phg_gradient_async(ctx, _vp(d_logl), _vp(d_grad)), ctx, "phg_gradient_async")


def phg_gradient_async_noalloc(ctx, d_logl: int, d_grad: int):
    _check(lib().phg_gradient_async_noalloc(ctx, _vp(d_logl), _vp(d_grad)), ctx,
           "phg_gradient_async_noalloc")


def phg_set_time_tree(ctx, heights, rates):
    h = _f64(heights)
    r = _f64(rates)
    _check(lib().phg_set_time_tree(ctx, _p(h), _p(r)), ctx, "phg_set_time_tree")


def phg_set_branch_sets(ctx, set_of, n_sets: int):
    if n_sets == 0:
        _check(lib().phg_set_branch_sets(ctx, None, 0), ctx, "phg_set_branch_sets")
        return
    a = _i32(set_of)
    _check(lib().phg_set_branch_sets(ctx, _p(a), int(n_sets)), ctx, "phg_set_branch_sets")


def phg_time_tree_gradient(ctx, n_tips: int, n_sets: int = 0):
    """Returns (logL, d_heights [2N-1], d_rates [2N-2], d_sets [n_sets] or None)."""
    E = 2 * n_tips - 2
    logl = ctypes.c_double()
    dh = np.empty(E + 1)
    dr = np.empty(E)
    ds = np.empty(n_sets) if n_sets else None
    _check(lib().phg_time_tree_gradient(ctx, ctypes.byref(logl), _p(dh), _p(dr),
                                        _p(ds) if ds is not None else None), ctx,
           "phg_time_tree_gradient")
    return logl.value, dh, dr, ds


def phg_gradient_branch_sets(ctx, n_sets: int):
    """Returns (logL, d_sets [n_sets])."""
    logl = ctypes.c_double()
    ds = np.empty(n_sets)
    _check(lib().phg_gradient_branch_sets(ctx, ctypes.byref(logl), _p(ds)), ctx,
           "phg_gradient_branch_sets")
    return logl.value, ds


def phg_get_schedule(ctx) -> int:
    v = ctypes.c_int()
    _check(lib().phg_get_schedule(ctx, ctypes.byref(v)), ctx, "phg_get_schedule")
    return v.value


def phg_schedule_info(ctx):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().phg_schedule_info(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), ctx,
           "phg_schedule_info")
    return a.value, b.value, c.value


def phg_profile_enable(ctx, on: bool):
    _check(lib().phg_profile_enable(ctx, 1 if on else 0), ctx, "phg_profile_enable")


def phg_profile_read(ctx):
    """Returns (ms[4] summed per kernel class, n_evals, launches[4] per eval)."""
    ms = np.zeros(PHG_PROF_CLASSES, np.float64)
    n = ctypes.c_int()
    launches = np.zeros(PHG_PROF_CLASSES, np.int32)
    _check(lib().phg_profile_read(ctx, _p(ms), ctypes.byref(n), _p(launches)), ctx,
           "phg_profile_read")
    return ms, n.value, launches


def phg_set_fp32_guard(ctx, threshold: float):
    _check(lib().phg_set_fp32_guard(ctx, float(threshold)), ctx, "phg_set_fp32_guard")


def phg_fp32_saturation(ctx) -> float:
    v = ctypes.c_double()
    _check(lib().phg_fp32_saturation(ctx, ctypes.byref(v)), ctx, "phg_fp32_saturation")
    return v.value


def phg_last_precision(ctx) -> int:
    v = ctypes.c_int()
    _check(lib().phg_last_precision(ctx, ctypes.byref(v)), ctx, "phg_last_precision")
    return v.value


def phg_set_table_budget(ctx, nbytes: int):
    _check(lib().phg_set_table_budget(ctx, int(nbytes)), ctx, "phg_set_table_budget")


def phg_table_slots(ctx) -> int:
    v = ctypes.c_int()
    _check(lib().phg_table_slots(ctx, ctypes.byref(v)), ctx, "phg_table_slots")
    return v.value


def phg_set_graphs(ctx, on: bool):
    _check(lib().phg_set_graphs(ctx, 1 if on else 0), ctx, "phg_set_graphs")


def phg_graph_stats(ctx):
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().phg_graph_stats(ctx, ctypes.byref(a), ctypes.byref(b)), ctx, "phg_graph_stats")
    return a.value, b.value


PHG_TUNE_ROW_BLOCKS = 0
PHG_TUNE_NARROW_UNITS = 1
PHG_TUNE_QUEUE_LAUNCHES = 2
PHG_TUNE_QUEUE_WAIT_US = 3


def phg_set_tuning(n_states: int, n_categories: int, prec: int, param: int, value: int):
    _check(lib().phg_set_tuning(n_states, n_categories, prec, param, value), None, "phg_set_tuning")


def phg_get_tuning(n_states: int, n_categories: int, prec: int, param: int) -> int:
    v = ctypes.c_int()
    _check(lib().phg_get_tuning(n_states, n_categories, prec, param, ctypes.byref(v)), None, "phg_get_tuning")
    return v.value


# ------------------------------------------------------------ serving

class phg_tree_desc(ctypes.Structure):
    _fields_ = [("n_tips", _c.c_int), ("n_patterns", _c.c_int), ("n_states", _c.c_int),
                ("n_categories", _c.c_int), ("prec", _c.c_int),
                ("parent", _ip), ("V", _dp), ("Vinv", _dp), ("lambda_", _dp), ("pi", _dp),
                ("rates", _dp), ("weights", _dp), ("codes", _ip), ("pattern_weights", _dp),
                ("per_category_eigen", _c.c_int), ("n_tip_vectors", _c.c_int), ("tip_vector_tips", _ip),
                ("tip_vectors", _dp)]


def _scheck(status: int, srv, where: str):
    if status != PHG_OK:
        msg = lib().phg_server_last_error(srv)
        raise PhgError(status, (msg or b"").decode(), where)


def phg_server_create(device: int, mem_budget_bytes: int, max_slots: int):
    out = _vp()
    _scheck(lib().phg_server_create(device, mem_budget_bytes, max_slots, ctypes.byref(out)), None,
            "phg_server_create")
    return out


def phg_server_destroy(srv):
    lib().phg_server_destroy(srv)


def phg_server_register_tree(srv, prob, prec) -> int:
    """Register a Problem-like object; returns the tree id."""
    keep = dict(parent=_i32(prob.parent), V=_f64(prob.V), Vinv=_f64(prob.Vinv), lam=_f64(prob.lam),
                pi=_f64(prob.pi), rates=_f64(prob.rates), weights=_f64(prob.weights),
                codes=_i32(prob.codes), pw=_f64(prob.pattern_weights))
    tv = getattr(prob, "tip_vectors", None) or {}
    tips = sorted(tv)
    keep["tv_tips"] = _i32(np.array(tips, np.int32)) if tips else None
    keep["tv"] = (_f64(np.concatenate([np.asarray(tv[t], np.float64).reshape(-1) for t in tips]))
                  if tips else None)
    d = phg_tree_desc(prob.n_tips, prob.n_patterns, prob.n_states, prob.n_categories, prec,
                      _p(keep["parent"]), _p(keep["V"]), _p(keep["Vinv"]), _p(keep["lam"]),
                      _p(keep["pi"]), _p(keep["rates"]), _p(keep["weights"]), _p(keep["codes"]),
                      _p(keep["pw"]), 1 if np.ndim(prob.V) == 3 else 0, len(tips),
                      _p(keep["tv_tips"]) if tips else None, _p(keep["tv"]) if tips else None)
    tid = ctypes.c_uint64()
    _scheck(lib().phg_server_register_tree(srv, ctypes.byref(d), ctypes.byref(tid)), srv,
            "phg_server_register_tree")
    return tid.value


def phg_server_submit(srv, tree_id: int, b) -> int:
    a = _f64(b)
    rid = ctypes.c_uint64()
    _scheck(lib().phg_server_submit(srv, tree_id, _p(a), ctypes.byref(rid)), srv, "phg_server_submit")
    return rid.value


def phg_server_poll(srv, req_id: int, n_branches: int):
    """Returns (done, logl, grad); raises PhgError for a finished failed request."""
    g = np.empty(n_branches, np.float64)
    v = ctypes.c_double()
    done = ctypes.c_int()
    _scheck(lib().phg_server_poll(srv, req_id, ctypes.byref(v), _p(g), ctypes.byref(done)), srv,
            "phg_server_poll")
    return bool(done.value), v.value, g


def phg_server_poll_timed(srv, req_id: int, n_branches: int):
    """Returns (done, logl, grad, t_submit_ns, t_done_ns) or raises PhgError."""
    g = np.empty(n_branches, np.float64)
    v = ctypes.c_double()
    done = ctypes.c_int()
    ts, td = ctypes.c_uint64(), ctypes.c_uint64()
    _scheck(lib().phg_server_poll_timed(srv, req_id, ctypes.byref(v), _p(g), ctypes.byref(done),
                                        ctypes.byref(ts), ctypes.byref(td)), srv, "phg_server_poll_timed")
    return bool(done.value), v.value, g, ts.value, td.value


def phg_server_wait(srv, req_id: int, n_branches: int):
    """Blocks until done; returns (logl, grad) or raises PhgError."""
    g = np.empty(n_branches, np.float64)
    v = ctypes.c_double()
    _scheck(lib().phg_server_wait(srv, req_id, ctypes.byref(v), _p(g)), srv, "phg_server_wait")
    return v.value, g


def phg_server_release_tree(srv, tree_id: int):
    _scheck(lib().phg_server_release_tree(srv, tree_id), srv, "phg_server_release_tree")


SERVER_STATS = ("completed", "steps", "launches", "resident_trees", "evictions", "peak_bytes",
                "queued", "in_flight")


def phg_server_busy(srv):
    """(kernel busy ns, wall ns) since the server's creation."""
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _scheck(lib().phg_server_busy(srv, ctypes.byref(a), ctypes.byref(b)), srv, "phg_server_busy")
    return a.value, b.value


def phg_server_stats(srv) -> dict:
    a = (ctypes.c_uint64 * 8)()
    _scheck(lib().phg_server_stats(srv, a), srv, "phg_server_stats")
    return dict(zip(SERVER_STATS, list(a)))


# ------------------------------------------------------------ convenience

def set_problem(h, prob):
    """Marshal every input of a synthetic Problem (or any object with the
    same fields) into context handle h."""
    phg_set_topology(h, prob.parent)
    phg_set_branch_lengths(h, prob.b)
    if np.ndim(prob.V) == 3:                 # one model per rate category
        phg_set_category_eigen(h, prob.V, prob.Vinv, prob.lam)
    else:
        phg_set_eigen(h, prob.V, prob.Vinv, prob.lam)
    phg_set_root_frequencies(h, prob.pi)
    phg_set_categories(h, prob.rates, prob.weights)
    phg_set_tip_states(h, prob.codes)
    for tip, vec in sorted((getattr(prob, "tip_vectors", None) or {}).items()):
        phg_set_tip_partials(h, tip, vec)
    phg_set_pattern_weights(h, prob.pattern_weights)


class Context:
    """Owns one phg_context; ``set_problem`` marshals every input of a
    synthetic Problem (or any object with the same fields)."""

    def __init__(self, n_tips, n_patterns, n_states, n_categories, prec=PHG_FP32_SCALED, device=0):
        self.n_tips = n_tips
        self.n_branches = 2 * n_tips - 2
        self.prec = prec
        self.handle = phg_create(n_tips, n_patterns, n_states, n_categories, prec, device)

    @classmethod
    def for_problem(cls, prob, prec=PHG_FP32_SCALED, device=0, schedule=PHG_SCHEDULE_AUTO):
        ctx = cls(prob.n_tips, prob.n_patterns, prob.n_states, prob.n_categories, prec, device)
        if schedule != PHG_SCHEDULE_AUTO:
            phg_set_schedule(ctx.handle, schedule)
        ctx.set_problem(prob)
        return ctx

    def set_problem(self, prob):
        set_problem(self.handle, prob)

    def gradient(self):
        return phg_gradient(self.handle, self.n_branches)

    def log_likelihood(self):
        return phg_log_likelihood(self.handle)

    def close(self):
        if self.handle:
            phg_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
