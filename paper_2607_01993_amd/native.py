"""ctypes binding of libsilh.so (the C ABI declared in include/silh.h).

Argument marshalling only: every step of the silhouette path runs in the HIP
library.  PyTorch provides device memory (through the allocator hooks of the
C ABI) and the stream the library enqueues on.  There is no fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsilh.so")

METRICS = {"eucl": 0, "cos": 1, "manh": 2, "canb": 3}
PRECS = {"fp32": 0, "bf16": 1, "fp8": 2, "fp32_valu": 3}
SAMPLERS = {"pps": 0, "uni": 1}
STATUS = {0: "SILH_OK", 1: "SILH_E_ARG", 2: "SILH_E_LABEL", 3: "SILH_E_K", 4: "SILH_E_STATE",
          5: "SILH_E_NOMEM", 6: "SILH_E_HIP", 7: "SILH_E_UNSUPPORTED"}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class SilhParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("prec", ctypes.c_int32), ("sampler", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("t", ctypes.c_int64), ("eps", ctypes.c_double),
                ("delta", ctypes.c_double), ("seed", ctypes.c_uint64), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_user", ctypes.c_void_p)]


class SilhSampleInfo(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int64), ("gid", ctypes.c_void_p),
                ("offsets_host", ctypes.POINTER(ctypes.c_int64)), ("p", ctypes.c_void_p),
                ("F0", ctypes.c_int64), ("f0_gid", ctypes.c_void_p), ("f0_W", ctypes.c_void_p),
                ("f0_offsets_host", ctypes.POINTER(ctypes.c_int64)), ("t", ctypes.c_int64)]


class SilhServerCfg(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("mode", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64)]


class SilhRequest(ctypes.Structure):
    _fields_ = [("dataset", ctypes.c_int32), ("k", ctypes.c_int32), ("labels", ctypes.c_void_p),
                ("metric", ctypes.c_int32), ("prec", ctypes.c_int32), ("sampler", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("t", ctypes.c_int64), ("delta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("m", ctypes.c_int64)]


class SilhResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("s_mean", ctypes.c_double),
                ("S", ctypes.c_int64), ("submit_ns", ctypes.c_int64), ("start_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("message", ctypes.c_char * 160)]


# name -> (restype, argtypes), exactly the symbols of include/*.h
SIGNATURES = {
    "silh_sample_init": (ctypes.c_int, [ctypes.POINTER(SilhParams), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "silh_pps_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "silh_weighted_sums": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "silh_scores": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double)]),
    "silh_exact": (ctypes.c_int, [ctypes.POINTER(SilhParams), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_double)]),
    "silh_exact_noalloc": (ctypes.c_int, [ctypes.POINTER(SilhParams), ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double)]),
    "silh_rows_for": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]),
    "silh_draw_rows": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "silh_scores_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "silh_exact_rows": (ctypes.c_int, [ctypes.POINTER(SilhParams), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "silh_coh_sep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
    "silh_set_tuning": (ctypes.c_int, [ctypes.c_int]),
    "silh_tuning_choice": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_int)]),
    "silh_sample_view": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SilhSampleInfo)]),
    "silh_philox_uniform": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]),
    "silh_prof_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "silh_prof_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "silh_prof_count": (ctypes.c_int, []),
    "silh_prof_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "silh_destroy": (None, [ctypes.c_void_p]),
    "silh_server_now_ns": (ctypes.c_int64, []),
    "silh_server_create": (ctypes.c_int, [ctypes.POINTER(SilhServerCfg), ctypes.POINTER(ctypes.c_void_p)]),
    "silh_server_add_dataset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32)]),
    "silh_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SilhRequest),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "silh_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(SilhResult)]),
    "silh_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "silh_server_destroy": (None, [ctypes.c_void_p]),
    "silh_server_launches": (ctypes.c_int64, [ctypes.c_void_p]),
    "silh_sweep": (ctypes.c_int, [ctypes.POINTER(SilhParams), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_uint64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32)]),
    "silh_graph_create": (ctypes.c_int, [ctypes.POINTER(SilhParams), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "silh_graph_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "silh_graph_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "silh_graph_choice": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "silh_graph_destroy": (None, [ctypes.c_void_p]),
    "silh_last_error": (ctypes.c_char_p, []),
    "silh_version": (ctypes.c_char_p, []),
}

_lib = None
_lock = threading.Lock()


def load_library(path: str = LIB_PATH):
    """Load libsilh.so (no GPU needed to load it).  Raises if it is missing."""
    global _lib
    with _lock:
        if _lib is None:
            # PyTorch ships its own HIP runtime under the same soname; load it
            # first so that the library and torch share one runtime (streams and
            # device memory are exchanged between them)
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            if not os.path.exists(path):
                raise RuntimeError(f"{path} is missing: build it with `python -m paper_2607_01993_amd.build`")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
        return _lib


class SilhError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def _check(status: int, where: str):
    if status != 0:
        msg = load_library().silh_last_error()
        raise SilhError(status, where, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# torch plumbing: device memory through the caching allocator, current stream
# ---------------------------------------------------------------------------
_TORCH = None


def _torch():
    global _TORCH
    if _TORCH is None:
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the silhouette library runs only on the MI355X")
        _TORCH = torch
    return _TORCH


_alloc_state = threading.local()


def _py_alloc(nbytes, user):
    torch = _torch()
    dev, stream = _alloc_state.target
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
    except Exception:   # out of memory: the library reports SILH_E_NOMEM
        return None


def _py_free(ptr, user):
    if ptr and _TORCH is not None:
        try:
            _TORCH.cuda.caching_allocator_delete(ptr)
        except Exception:   # interpreter shutdown: the process frees device memory itself
            pass


_ALLOC_CB = ALLOC_FN(_py_alloc)
_FREE_CB = FREE_FN(_py_free)


class _Target:
    def __init__(self, device, stream):
        self.t = (device, stream)

    def __enter__(self):
        self.prev = getattr(_alloc_state, "target", None)
        _alloc_state.target = self.t

    def __exit__(self, *a):
        _alloc_state.target = self.prev


def _params(n, d, k, metric, prec, sampler, t, eps, delta, seed, use_torch_alloc=True):
    p = SilhParams()
    p.n, p.d, p.k = int(n), int(d), int(k)
    p.metric = METRICS[metric] if isinstance(metric, str) else int(metric)
    p.prec = PRECS[prec] if isinstance(prec, str) else int(prec)
    p.sampler = SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler)
    p.reserved0 = 0
    p.t = int(t)
    p.eps = float(eps)
    p.delta = float(delta)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    if use_torch_alloc:
        p.alloc, p.free = _ALLOC_CB, _FREE_CB
    else:
        p.alloc, p.free = ALLOC_FN(), FREE_FN()
    p.alloc_user = None
    return p


def _check_inputs(X, labels):
    torch = _torch()
    if not (X.is_cuda and labels.is_cuda):
        raise ValueError("X and labels must be device tensors")
    if X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous float32 [n, d] tensor")
    if labels.dtype != torch.int32 or labels.dim() != 1 or labels.shape[0] != X.shape[0] \
            or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous int32 [n] tensor")


class Context:
    """A silh_ctx plus the tensors it references."""

    def __init__(self, ptr, X, labels, params, device, stream):
        self.ptr = ptr
        self.X, self.labels = X, labels
        self.params = params
        self.device, self.stream = device, stream
        self.n, self.d, self.k = params.n, params.d, params.k

    def target(self):
        return _Target(self.device, self.stream)

    def __del__(self):
        try:
            silh_destroy(self)
        except Exception:
            pass


def _stream_handle(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s, ctypes.c_void_p(s.cuda_stream)


def silh_sample_init(X, labels, k, metric="eucl", prec="fp32", sampler="pps", t=0, eps=0.0,
                     delta=0.01, seed=0, stream=None, use_torch_alloc=True) -> Context:
    lib = load_library()
    _check_inputs(X, labels)
    s, sh = _stream_handle(stream)
    p = _params(X.shape[0], X.shape[1], k, metric, prec, sampler, t, eps, delta, seed, use_torch_alloc)
    out = ctypes.c_void_p()
    with _Target(X.device.index, s):
        _check(lib.silh_sample_init(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()),
                                    ctypes.c_void_p(labels.data_ptr()), sh, ctypes.byref(out)),
               "silh_sample_init")
    return Context(out, X, labels, p, X.device.index, s)


def silh_pps_sample(ctx: Context):
    import numpy as np
    lib = load_library()
    S = ctypes.c_int64()
    per = (ctypes.c_int64 * ctx.k)()
    with ctx.target():
        _check(lib.silh_pps_sample(ctx.ptr, ctypes.byref(S), per), "silh_pps_sample")
    return int(S.value), np.frombuffer(per, dtype=np.int64).copy()


def silh_weighted_sums(ctx: Context, out=None):
    torch = _torch()
    lib = load_library()
    W = out if out is not None else torch.empty((ctx.n, ctx.k), dtype=torch.float32, device=ctx.X.device)
    with ctx.target():
        _check(lib.silh_weighted_sums(ctx.ptr, ctypes.c_void_p(W.data_ptr())), "silh_weighted_sums")
    return W


def silh_scores(ctx: Context, a=True, b=True, s=True, mean=True):
    torch = _torch()
    lib = load_library()
    dev = ctx.X.device
    outs = {name: torch.empty(ctx.n, dtype=torch.float32, device=dev) if want else None
            for name, want in (("a", a), ("b", b), ("s", s))}
    m = ctypes.c_double()
    ptr = [ctypes.c_void_p(outs[x].data_ptr()) if outs[x] is not None else ctypes.c_void_p()
           for x in ("a", "b", "s")]
    with ctx.target():
        _check(lib.silh_scores(ctx.ptr, *ptr, ctypes.byref(m) if mean else None), "silh_scores")
    res = {x: v for x, v in outs.items() if v is not None}
    if mean:
        res["mean"] = m.value
    return res


def silh_exact(X, labels, k, metric="eucl", prec="fp32", stream=None, a=True, b=True, s=True,
               mean=True, use_torch_alloc=True):
    torch = _torch()
    lib = load_library()
    _check_inputs(X, labels)
    st, sh = _stream_handle(stream)
    p = _params(X.shape[0], X.shape[1], k, metric, prec, "pps", 1, 0.0, 0.5, 0, use_torch_alloc)
    outs = {name: torch.empty(X.shape[0], dtype=torch.float32, device=X.device) if want else None
            for name, want in (("a", a), ("b", b), ("s", s))}
    ptr = [ctypes.c_void_p(outs[x].data_ptr()) if outs[x] is not None else ctypes.c_void_p()
           for x in ("a", "b", "s")]
    m = ctypes.c_double()
    with _Target(X.device.index, st):
        _check(lib.silh_exact(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()),
                              ctypes.c_void_p(labels.data_ptr()), sh, *ptr,
                              ctypes.byref(m) if mean else None), "silh_exact")
    res = {x: v for x, v in outs.items() if v is not None}
    if mean:
        res["mean"] = m.value
    return res


def silh_exact_noalloc(X, labels, k, metric="eucl", prec="fp32", stream=None, a=True, b=True, s=True,
                       mean=True):
    """silh_exact with the library's buffers in its static device array (no
    device allocation by the library; the outputs are allocated here)."""
    torch = _torch()
    lib = load_library()
    _check_inputs(X, labels)
    st, sh = _stream_handle(stream)
    p = _params(X.shape[0], X.shape[1], k, metric, prec, "pps", 1, 0.0, 0.5, 0, False)
    outs = {name: torch.empty(X.shape[0], dtype=torch.float32, device=X.device) if want else None
            for name, want in (("a", a), ("b", b), ("s", s))}
    ptr = [ctypes.c_void_p(outs[x].data_ptr()) if outs[x] is not None else ctypes.c_void_p()
           for x in ("a", "b", "s")]
    m = ctypes.c_double()
    with _Target(X.device.index, st):
        _check(lib.silh_exact_noalloc(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()),
                                      ctypes.c_void_p(labels.data_ptr()), sh, *ptr,
                                      ctypes.byref(m) if mean else None), "silh_exact_noalloc")
    res = {x: v for x, v in outs.items() if v is not None}
    if mean:
        res["mean"] = m.value
    return res


def silh_rows_for(eps, delta) -> int:
    """m = ceil((2/eps^2) ln(2/delta)) of the subsampled estimators."""
    lib = load_library()
    m = ctypes.c_int64()
    _check(lib.silh_rows_for(float(eps), float(delta), ctypes.byref(m)), "silh_rows_for")
    return int(m.value)


def silh_draw_rows(seed, n, m, stream=None):
    """m independent uniform row indices in [0, n) (device int32)."""
    torch = _torch()
    lib = load_library()
    st, sh = _stream_handle(stream)
    rows = torch.empty(max(int(m), 1), dtype=torch.int32, device="cuda")[:int(m)]
    _check(lib.silh_draw_rows(int(seed) & 0xFFFFFFFFFFFFFFFF, int(n), int(m),
                              ctypes.c_void_p(rows.data_ptr()), sh), "silh_draw_rows")
    return rows


def _rows_outputs(rows, a, b, s):
    torch = _torch()
    if rows.dtype != torch.int32 or rows.dim() != 1 or not rows.is_cuda or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous int32 device vector")
    m = rows.shape[0]
    outs = {name: torch.empty(m, dtype=torch.float32, device=rows.device) if want else None
            for name, want in (("a", a), ("b", b), ("s", s))}
    ptr = [ctypes.c_void_p(outs[x].data_ptr()) if outs[x] is not None else ctypes.c_void_p()
           for x in ("a", "b", "s")]
    return m, outs, ptr


def silh_scores_rows(ctx: Context, rows, a=True, b=True, s=True, mean=True):
    """gl-pps-s / gl-uni-s (Eq. 10): Phase-2 scores of the entries of rows."""
    lib = load_library()
    m, outs, ptr = _rows_outputs(rows, a, b, s)
    mv = ctypes.c_double()
    with ctx.target():
        _check(lib.silh_scores_rows(ctx.ptr, ctypes.c_void_p(rows.data_ptr()), m, *ptr,
                                    ctypes.byref(mv) if mean else None), "silh_scores_rows")
    res = {x: v for x, v in outs.items() if v is not None}
    if mean:
        res["mean"] = mv.value
    return res


def silh_exact_rows(X, labels, k, rows, metric="eucl", prec="fp32", stream=None, a=True, b=True, s=True,
                    mean=True, use_torch_alloc=True):
    """gl-s (Eq. 8): exact scores of the entries of rows."""
    lib = load_library()
    _check_inputs(X, labels)
    st, sh = _stream_handle(stream)
    p = _params(X.shape[0], X.shape[1], k, metric, prec, "pps", 1, 0.0, 0.5, 0, use_torch_alloc)
    m, outs, ptr = _rows_outputs(rows, a, b, s)
    mv = ctypes.c_double()
    with _Target(X.device.index, st):
        _check(lib.silh_exact_rows(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()),
                                   ctypes.c_void_p(labels.data_ptr()), ctypes.c_void_p(rows.data_ptr()), m,
                                   sh, *ptr, ctypes.byref(mv) if mean else None), "silh_exact_rows")
    res = {x: v for x, v in outs.items() if v is not None}
    if mean:
        res["mean"] = mv.value
    return res


def silh_coh_sep(ctx: Context, W_hat=None):
    """Estimated cohesion and separation (Appendix B); W_hat from
    silh_weighted_sums, or None to let the library compute it."""
    lib = load_library()
    coh, sep = ctypes.c_double(), ctypes.c_double()
    wp = ctypes.c_void_p(W_hat.data_ptr()) if W_hat is not None else ctypes.c_void_p()
    with ctx.target():
        _check(lib.silh_coh_sep(ctx.ptr, wp, ctypes.byref(coh), ctypes.byref(sep)), "silh_coh_sep")
    return {"coh": coh.value, "sep": sep.value}


def gl_s(X, labels, k, m, seed, metric="eucl", prec="fp32"):
    """Eq. 8: mean of the exact silhouette over m uniform draws of rows."""
    rows = silh_draw_rows(seed, X.shape[0], m)
    res = silh_exact_rows(X, labels, k, rows, metric, prec)
    res["rows"] = rows
    return res


def gl_pps_s(X, labels, k, m, t, seed, rows_seed, metric="eucl", prec="fp32", sampler="pps", delta=0.01):
    """Eq. 10 (gl-pps-s; gl-uni-s with sampler="uni"): Phase 1, then the
    Phase-2 scores of m uniform draws of rows and their mean."""
    ctx = silh_sample_init(X, labels, k, metric, prec, sampler, t=t, delta=delta, seed=seed)
    silh_pps_sample(ctx)
    rows = silh_draw_rows(rows_seed, X.shape[0], m)
    res = silh_scores_rows(ctx, rows)
    res["rows"] = rows
    silh_destroy(ctx)
    return res


def silh_set_tuning(mode):
    """0 built-in block shape, 1 autotune (default), 2 / 3 / 4 force shape 1
    (one 32-element block per wave), 2 (two blocks) or 3 (one block, the
    other number of tiles per LDS stage) of the matrix-core Phase 2."""
    _check(load_library().silh_set_tuning(int(mode)), "silh_set_tuning")


def silh_tuning_choice(metric, prec, d, S_pad):
    pb = ctypes.c_int()
    _check(load_library().silh_tuning_choice(METRICS[metric] if isinstance(metric, str) else int(metric),
                                             PRECS[prec] if isinstance(prec, str) else int(prec), int(d),
                                             int(S_pad), ctypes.byref(pb)), "silh_tuning_choice")
    return int(pb.value)


class _DevArray:
    """Zero-copy wrapper so torch can view library-owned device memory."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr or 0), False), "version": 2}


def silh_sample_view(ctx: Context) -> dict:
    """Copies of the Phase-1 result: sample ids, offsets, p, initial sample."""
    import numpy as np
    torch = _torch()
    lib = load_library()
    info = SilhSampleInfo()
    _check(lib.silh_sample_view(ctx.ptr, ctypes.byref(info)), "silh_sample_view")
    torch.cuda.synchronize()
    k = ctx.k

    def dev(ptr, count, typestr):
        if count == 0:
            return torch.empty(0, dtype=torch.int64 if typestr == "<i8" else torch.float64)
        return torch.as_tensor(_DevArray(ptr, (count,), typestr), device=ctx.X.device).clone().cpu()

    return {
        "S": int(info.S), "t": int(info.t),
        "gid": dev(info.gid, info.S, "<i8").numpy(),
        "offsets": np.array([info.offsets_host[j] for j in range(k + 1)], dtype=np.int64),
        "p": dev(info.p, ctx.n, "<f8").numpy(),
        "F0": int(info.F0),
        "f0_gid": dev(info.f0_gid, info.F0, "<i8").numpy(),
        "f0_W": dev(info.f0_W, info.F0, "<f8").numpy(),
        "f0_offsets": np.array([info.f0_offsets_host[j] for j in range(k + 1)], dtype=np.int64),
    }


def silh_philox_uniform(seed, gid0, count, stream_id, stream=None):
    torch = _torch()
    lib = load_library()
    st, sh = _stream_handle(stream)
    out = torch.empty(int(count), dtype=torch.float64, device="cuda")
    _check(lib.silh_philox_uniform(int(seed) & 0xFFFFFFFFFFFFFFFF, int(gid0), int(count), int(stream_id),
                                   ctypes.c_void_p(out.data_ptr()), sh), "silh_philox_uniform")
    return out


def silh_prof_enable(ctx: Context, on=True):
    """on: True / 1 = every kernel, 2 = the Phase-2 launches only, False / 0 = off."""
    mode = int(on) if not isinstance(on, bool) else (1 if on else 0)
    _check(load_library().silh_prof_enable(ctx.ptr, mode), "silh_prof_enable")


def silh_prof_reset(ctx: Context):
    _check(load_library().silh_prof_reset(ctx.ptr), "silh_prof_reset")


def silh_prof_get(ctx: Context) -> dict:
    lib = load_library()
    res = {}
    for i in range(lib.silh_prof_count()):
        name = ctypes.c_char_p()
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib.silh_prof_get(ctx.ptr, i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)),
               "silh_prof_get")
        res[name.value.decode()] = (int(cnt.value), float(ms.value))
    return res


def silh_destroy(ctx: Context):
    if ctx is not None and ctx.ptr:
        lib = load_library()
        with ctx.target():
            lib.silh_destroy(ctx.ptr)
        ctx.ptr = None


def version() -> str:
    return load_library().silh_version().decode()


def silh_sweep(X, labels, ks, metric="eucl", prec="bf16", sampler="pps", t=128, delta=0.01, seed=0, m=0,
               workers=4, hbm_budget_bytes=64 << 30, stream=None):
    """s_hat_2 (m = 0) or the Eq. 10 mean over m row draws of K clusterings
    (labels [K, n] int32 device, ks their k) and the index of the best one."""
    import numpy as np
    torch = _torch()
    lib = load_library()
    if labels.dtype != torch.int32 or labels.dim() != 2 or labels.shape[1] != X.shape[0] \
            or not labels.is_contiguous() or not labels.is_cuda:
        raise ValueError("labels must be a contiguous int32 [K, n] device tensor")
    K = labels.shape[0]
    ksa = (ctypes.c_int32 * K)(*[int(v) for v in ks])
    means = (ctypes.c_double * K)()
    best = ctypes.c_int32()
    st, sh = _stream_handle(stream)
    p = _params(X.shape[0], X.shape[1], 2, metric, prec, sampler, t, 0.0, delta, seed, use_torch_alloc=False)
    _check(lib.silh_sweep(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(labels.data_ptr()), ksa,
                          K, int(m), int(workers), int(hbm_budget_bytes), sh, means, ctypes.byref(best)),
           "silh_sweep")
    return {"means": np.frombuffer(means, dtype=np.float64).copy(), "best": int(best.value)}


class SilhGraphInfo(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("sample_cap", ctypes.c_int64), ("f0_cap", ctypes.c_int64),
                ("bytes", ctypes.c_int64)]


class SweepGraph:
    """K clusterings of one dataset captured into one HIP graph
    (include/silh_graph.h).  labels is a contiguous int32 [K, n] device tensor
    whose contents are read at every run(), so new label sets may be written
    into it between runs."""

    def __init__(self, X, labels, ks, metric="eucl", prec="bf16", sampler="pps", t=128, delta=0.01, seed=0,
                 chains=4, sample_cap=0.0, stream=None):
        torch = _torch()
        lib = load_library()
        if labels.dtype != torch.int32 or labels.dim() != 2 or labels.shape[1] != X.shape[0] \
                or not labels.is_contiguous() or not labels.is_cuda:
            raise ValueError("labels must be a contiguous int32 [K, n] device tensor")
        if X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous() or not X.is_cuda:
            raise ValueError("X must be a contiguous float32 [n, d] device tensor")
        self.K = labels.shape[0]
        self.X, self.labels = X, labels  # referenced by the graph until close()
        ksa = (ctypes.c_int32 * self.K)(*[int(v) for v in ks])
        _, sh = _stream_handle(stream)
        p = _params(X.shape[0], X.shape[1], 2, metric, prec, sampler, t, 0.0, delta, seed, use_torch_alloc=False)
        out = ctypes.c_void_p()
        _check(lib.silh_graph_create(ctypes.byref(p), ctypes.c_void_p(X.data_ptr()),
                                     ctypes.c_void_p(labels.data_ptr()), ksa, self.K, int(chains),
                                     float(sample_cap), sh, ctypes.byref(out)), "silh_graph_create")
        self.ptr = out

    def run(self, stream=None):
        import numpy as np
        lib = load_library()
        _, sh = _stream_handle(stream)
        means = (ctypes.c_double * self.K)()
        status = (ctypes.c_int32 * self.K)()
        best, reruns = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.silh_graph_run(self.ptr, sh, means, status, ctypes.byref(best), ctypes.byref(reruns)),
               "silh_graph_run")
        return {"means": np.frombuffer(means, dtype=np.float64).copy(),
                "status": [STATUS.get(int(v), int(v)) for v in status], "best": int(best.value),
                "reruns": int(reruns.value)}

    def choice(self, i):
        """(shape id captured for clustering i, padded sample size it was tuned on)"""
        shape, S = ctypes.c_int32(), ctypes.c_int64()
        _check(load_library().silh_graph_choice(self.ptr, int(i), ctypes.byref(shape), ctypes.byref(S)),
               "silh_graph_choice")
        return int(shape.value), int(S.value)

    def info(self):
        out = SilhGraphInfo()
        _check(load_library().silh_graph_get_info(self.ptr, ctypes.byref(out)), "silh_graph_get_info")
        return {f: int(getattr(out, f)) for f, _ in SilhGraphInfo._fields_}

    def close(self):
        if self.ptr:
            load_library().silh_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# serving runtime (include/silh_server.h)
# ---------------------------------------------------------------------------
class Server:
    """Resident datasets, a request queue with a device-memory budget, and
    worker threads with their own streams (all in the HIP library)."""

    def __init__(self, workers=4, hbm_budget_bytes=64 << 30, batched=True):
        _torch()
        lib = load_library()
        cfg = SilhServerCfg(int(workers), 0 if batched else 1, int(hbm_budget_bytes))
        out = ctypes.c_void_p()
        _check(lib.silh_server_create(ctypes.byref(cfg), ctypes.byref(out)), "silh_server_create")
        self.ptr = out
        self._keep = {}       # device tensors that must outlive the requests using them
        self._datasets = []

    def add_dataset(self, X):
        torch = _torch()
        if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
            raise ValueError("X must be a contiguous float32 [n, d] device tensor")
        did = ctypes.c_int32()
        _check(load_library().silh_server_add_dataset(self.ptr, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                                      X.shape[1], ctypes.byref(did)), "silh_server_add_dataset")
        self._datasets.append(X)
        return int(did.value)

    def submit(self, dataset, labels, k, metric="eucl", prec="bf16", sampler="pps", t=256, delta=0.01, seed=0, m=0):
        torch = _torch()
        if not labels.is_cuda or labels.dtype != torch.int32 or not labels.is_contiguous():
            raise ValueError("labels must be a contiguous int32 device tensor")
        req = SilhRequest(int(dataset), int(k), ctypes.c_void_p(labels.data_ptr()),
                          METRICS[metric] if isinstance(metric, str) else int(metric),
                          PRECS[prec] if isinstance(prec, str) else int(prec),
                          SAMPLERS[sampler] if isinstance(sampler, str) else int(sampler), 0, int(t),
                          float(delta), int(seed) & 0xFFFFFFFFFFFFFFFF, int(m))
        tk = ctypes.c_int64()
        _check(load_library().silh_server_submit(self.ptr, ctypes.byref(req), ctypes.byref(tk)),
               "silh_server_submit")
        self._keep[int(tk.value)] = labels
        return int(tk.value)

    def wait(self, ticket):
        res = SilhResult()
        _check(load_library().silh_server_wait(self.ptr, int(ticket), ctypes.byref(res)), "silh_server_wait")
        self._keep.pop(int(ticket), None)
        return {"status": STATUS.get(res.status, res.status), "s_mean": res.s_mean, "S": int(res.S),
                "submit_ns": int(res.submit_ns), "start_ns": int(res.start_ns), "done_ns": int(res.done_ns),
                "message": res.message.decode(errors="replace")}

    def drain(self):
        _check(load_library().silh_server_drain(self.ptr), "silh_server_drain")

    def launches(self):
        """Shared Phase-2 launches issued so far."""
        return int(load_library().silh_server_launches(self.ptr))

    @staticmethod
    def now_ns():
        return int(load_library().silh_server_now_ns())

    def close(self):
        if self.ptr:
            load_library().silh_server_destroy(self.ptr)
            self.ptr = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
