"""MI355X GraphGuess sweep: Python binding of the C ABI in include/gg.h.

This module only marshals arguments: every step of the sweep runs in the HIP
kernels of libgg.so. PyTorch provides device memory (the library allocates
through torch's caching allocator, gg_set_allocator) and streams. torch is
imported before the library is loaded so that the process holds a single HIP
runtime (torch's).

If libgg.so is missing, loading fails with an error: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgg.so")

APP = {"pr": 0, "sssp": 1, "cc": 2, "ppr": 3, "bp": 4}
POLICY = {"exact": 0, "sp": 1, "sms": 2, "gg": 3, "learned": 4}
STEP_KIND = {0: "approx", 1: "accurate", 2: "full", 3: "partial"}
MLP_IN, MLP_HIDDEN, MLP_PARAMS = 8, 64, 4801
STOP = {"fixed_iters": 0, "fixed_point": 1}
INFLUENCE = {"prefix": 0, "total": 1, "push": 2}
MASK = {"replace": 0, "union": 1}
DANGLING = {"uniform": 0, "none": 1}
CSR_DEVICE_PTRS = 0x1
CSR_SKIP_VALIDATE = 0x2
OUT_HOST = 0x1
INF = 0xFFFFFFFF

STATUS = {0: "GG_OK", -1: "GG_E_INVAL", -2: "GG_E_RANGE", -3: "GG_E_NOMEM", -4: "GG_E_DEVICE",
          -5: "GG_E_UNSUPPORTED", -6: "GG_E_STATE"}


class GGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code


class CsrDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class AppParams(ctypes.Structure):
    _fields_ = [("app", ctypes.c_int32), ("damping", ctypes.c_double), ("iters", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("source", ctypes.c_int32), ("dangling", ctypes.c_int32),
                ("pr_degree", ctypes.c_int32), ("coupling", ctypes.c_double), ("prior", ctypes.c_void_p)]


class UpdateBatch(ctypes.Structure):
    _fields_ = [("n_delete", ctypes.c_int64), ("del_src", ctypes.c_void_p), ("del_dst", ctypes.c_void_p),
                ("n_insert", ctypes.c_int64), ("ins_src", ctypes.c_void_p), ("ins_dst", ctypes.c_void_p),
                ("ins_weight", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


UPDATE_DEVICE_PTRS = 0x1


def _batch(del_src=(), del_dst=(), ins_src=(), ins_dst=(), ins_weight=None):
    """gg_update_batch over host int32 copies (returned with the struct, which
    points into them). Device tensors (int32, contiguous) are passed as
    device pointers."""
    arrs = [del_src, del_dst, ins_src, ins_dst]
    dev = any(isinstance(a, torch.Tensor) and a.is_cuda for a in arrs + [ins_weight])
    if dev:
        keep = [None if a is None else a.to(device="cuda", dtype=torch.int32).contiguous() for a in arrs + [ins_weight]]
        ptr = lambda a: None if a is None or a.numel() == 0 else a.data_ptr()
        cnt = lambda a: 0 if a is None else int(a.numel())
    else:
        keep = [None if a is None else np.ascontiguousarray(np.asarray(a), dtype=np.int32) for a in arrs + [ins_weight]]
        ptr = lambda a: None if a is None or a.size == 0 else a.ctypes.data
        cnt = lambda a: 0 if a is None else int(a.size)
    ds, dd, is_, id_, iw = keep
    if cnt(ds) != cnt(dd) or cnt(is_) != cnt(id_) or (iw is not None and cnt(iw) != cnt(is_)):
        raise ValueError("source, destination and weight lists must have equal lengths")
    b = UpdateBatch(cnt(ds), ptr(ds), ptr(dd), cnt(is_), ptr(is_), ptr(id_), ptr(iw),
                    UPDATE_DEVICE_PTRS if dev else 0)
    return b, keep


class Policy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("alpha", ctypes.c_int32), ("theta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("influence", ctypes.c_int32), ("mask_update", ctypes.c_int32),
                ("stop", ctypes.c_int32), ("mlp", ctypes.c_void_p), ("tau", ctypes.c_float), ("rho", ctypes.c_double),
                ("fallback_k", ctypes.c_int32), ("audit", ctypes.c_int32), ("trace", ctypes.c_void_p),
                ("label_eps", ctypes.c_float), ("decoupled", ctypes.c_int32), ("alpha0", ctypes.c_int32),
                ("theta0", ctypes.c_double), ("vstatus", ctypes.c_int32), ("eps", ctypes.c_double)]


class RunStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("supersteps", ctypes.c_int32), ("edges_gathered", ctypes.c_int64),
                ("active_edges", ctypes.c_int64), ("device_ms", ctypes.c_double), ("edges_processed", ctypes.c_int64),
                ("sparse_iterations", ctypes.c_int32), ("partial_supersteps", ctypes.c_int32),
                ("selected_total", ctypes.c_int64), ("audit_positives", ctypes.c_int64), ("audit_hits", ctypes.c_int64),
                ("audit_selected", ctypes.c_int64)]


class StepInfo(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("accurate", ctypes.c_int32), ("superstep", ctypes.c_int32),
                ("edges", ctypes.c_int64), ("changed", ctypes.c_int64), ("active_edges", ctypes.c_int64),
                ("edges_processed", ctypes.c_int64), ("sparse", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("selected", ctypes.c_int64)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("edges", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("small_max", ctypes.c_int32), ("small_team", ctypes.c_int32), ("wave_max", ctypes.c_int32),
                ("hub_chunk", ctypes.c_int32), ("seg_enable", ctypes.c_int32), ("seg_vertices", ctypes.c_int32),
                ("frontier_enable", ctypes.c_int32), ("frontier_div", ctypes.c_int32)]

TUNING_FIELDS = [f[0] for f in Tuning._fields_]


# Every symbol the header declares, with its ctypes signature.
_VP = ctypes.c_void_p
SIGNATURES = {
    "gg_version": (ctypes.c_int, []),
    "gg_set_allocator": (ctypes.c_int, [_VP, _VP, _VP]),
    "gg_live_objects": (ctypes.c_int64, []),
    "gg_last_error": (ctypes.c_char_p, []),
    "gg_graph_load_csr": (ctypes.c_int, [ctypes.POINTER(CsrDesc), _VP, ctypes.POINTER(_VP)]),
    "gg_graph_set_stream": (ctypes.c_int, [_VP, _VP]),
    "gg_graph_free": (None, [_VP]),
    "gg_exact_run": (ctypes.c_int, [_VP, ctypes.POINTER(AppParams), _VP, ctypes.c_uint32, ctypes.POINTER(RunStats)]),
    "gg_exact_run_noalloc": (ctypes.c_int, [_VP, ctypes.POINTER(AppParams), _VP, ctypes.POINTER(RunStats)]),
    "gg_approx_run": (ctypes.c_int, [_VP, ctypes.POINTER(AppParams), ctypes.c_double, ctypes.POINTER(Policy), _VP,
                                     ctypes.c_uint32, ctypes.POINTER(RunStats)]),
    "gg_run_begin": (ctypes.c_int, [_VP, ctypes.POINTER(AppParams), ctypes.c_double, ctypes.POINTER(Policy),
                                    ctypes.POINTER(_VP)]),
    "gg_run_step": (ctypes.c_int, [_VP, ctypes.POINTER(StepInfo)]),
    "gg_run_values": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32]),
    "gg_run_mask": (ctypes.c_int, [_VP, _VP]),
    "gg_run_vstatus": (ctypes.c_int, [_VP, _VP]),
    "gg_run_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(RunStats)]),
    "gg_run_end": (None, [_VP]),
    "gg_graph_update": (ctypes.c_int, [_VP, _VP]),
    "gg_graph_set_capture": (ctypes.c_int, [_VP, ctypes.c_int]),
    "gg_run_update": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP]),
    "gg_graph_get_csr": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "gg_graph_num_arcs": (ctypes.c_int64, [_VP]),
    "gg_graph_get_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(Tuning)]),
    "gg_graph_set_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(Tuning)]),
    "gg_batch_run": (ctypes.c_int, [_VP, ctypes.POINTER(AppParams), ctypes.c_int32, _VP, ctypes.c_double,
                                    ctypes.POINTER(Policy), _VP, ctypes.c_uint32, ctypes.POINTER(RunStats)]),
    "gg_graph_autotune": (ctypes.c_int, [_VP, ctypes.POINTER(AppParams), ctypes.c_double, ctypes.POINTER(Policy),
                                         ctypes.c_int32, _VP, ctypes.c_int32, ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_double)]),
    "gg_graph_set_parts": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP]),
    "gg_graph_set_wait_limit": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "gg_graph_set_profiling": (ctypes.c_int, [_VP, ctypes.c_int]),
    "gg_graph_get_profile": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(KernelProfile)]),
    "gg_run_features": (ctypes.c_int, [_VP, _VP]),
    "gg_run_selection": (ctypes.c_int, [_VP, _VP, _VP]),
    "gg_run_labels": (ctypes.c_int, [_VP, _VP]),
    "gg_run_state_size": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "gg_run_export_state": (ctypes.c_int, [_VP, _VP, ctypes.c_int64]),
    "gg_run_import_state": (ctypes.c_int, [_VP, _VP, ctypes.c_int64]),
    "gg_mlp_create": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(_VP)]),
    "gg_mlp_free": (None, [_VP]),
    "gg_mlp_set_weights": (ctypes.c_int, [_VP, _VP]),
    "gg_mlp_get_weights": (ctypes.c_int, [_VP, _VP]),
    "gg_mlp_forward": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP]),
    "gg_mlp_loss_grad": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_float, _VP]),
    "gg_mlp_adam_step": (ctypes.c_int, [_VP, _VP, ctypes.c_float]),
    "gg_mlp_train": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_uint64, _VP]),
    "gg_trace_create": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(_VP)]),
    "gg_trace_free": (None, [_VP]),
    "gg_trace_clear": (ctypes.c_int, [_VP]),
    "gg_trace_info": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "gg_trace_export": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _VP, _VP]),
}

PROFILE_KIND = {"gather_exact": 0, "gather_approx": 1, "superstep": 2, "push": 3, "partial": 4}

_lib = None

# Device allocator callbacks (gg_set_allocator): C function pointers made
# from Python functions; the module keeps them alive.
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator = None  # (ALLOC_FN, FREE_FN) installed, or None for hipMalloc


def _torch_alloc(nbytes, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes))
    except Exception:  # out of memory: the library reports GG_E_NOMEM
        return None


def _torch_free(ptr, ctx):
    try:
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


def set_allocator(alloc=None, free=None):
    """gg_set_allocator with Python callables alloc(nbytes) -> int address
    (0 or None on failure) and free(address); both None restores hipMalloc.
    "torch" for alloc selects torch's caching allocator (the default once the
    library is loaded). Only while no graph, network or trace exists."""
    global _allocator
    if alloc == "torch":
        pair = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))
    elif alloc is None and free is None:
        pair = None
    else:
        pair = (ALLOC_FN(lambda nb, ctx: alloc(int(nb)) or None), FREE_FN(lambda p, ctx: free(int(p))))
    if pair is None:
        _check(lib().gg_set_allocator(None, None, None))
    else:
        _check(lib().gg_set_allocator(ctypes.cast(pair[0], _VP), ctypes.cast(pair[1], _VP), None))
    _allocator = pair


def live_objects():
    """gg_live_objects: graphs, networks and traces the library holds."""
    return int(lib().gg_live_objects())


# Objects that hold library handles, closed at interpreter exit while torch
# (whose allocator frees their memory) is still alive.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    objs = list(_live)
    # step-API runs first: freeing a graph also ends its run
    for obj in sorted(objs, key=lambda o: not isinstance(o, Run)):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    """Load libgg.so (built by __graft_entry__.build() / _build.py). Raises if
    missing. Device memory of the library's objects then comes from torch's
    caching allocator."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgg.so is not built (%s); run paper_2104_10039_amd/_build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        set_allocator("torch")
    return _lib


def _check(code: int):
    if code < 0:
        raise GGError(code, lib().gg_last_error().decode())
    return code


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    return x.ctypes.data


def _value_dtype(app: str):
    return {"pr": torch.float32, "ppr": torch.float32, "bp": torch.float32, "sssp": torch.int32,
            "cc": torch.int32}[app]


@dataclass
class Stats:
    iterations: int
    supersteps: int
    edges_gathered: int
    active_edges: int
    device_ms: float
    edges_processed: int
    sparse_iterations: int
    partial_supersteps: int = 0
    selected_total: int = 0
    audit_positives: int = 0
    audit_hits: int = 0
    audit_selected: int = 0


def _stats(s: RunStats) -> Stats:
    return Stats(s.iterations, s.supersteps, s.edges_gathered, s.active_edges, s.device_ms, s.edges_processed,
                 s.sparse_iterations, s.partial_supersteps, s.selected_total, s.audit_positives, s.audit_hits,
                 s.audit_selected)


PR_DEGREE = {"full": 0, "active": 1}


def _app_params(app, damping=0.85, iters=20, max_iters=1 << 20, source=0, dangling="uniform", pr_degree="full",
                coupling=0.0, prior=None):
    """prior: None or a float32 device tensor (see _prior_dev), read during the call."""
    return AppParams(APP[app], damping, iters, max_iters, source, DANGLING[dangling], PR_DEGREE[pr_degree],
                     float(coupling), None if prior is None else prior.data_ptr())


def _prior_dev(prior, n):
    """BP prior log-odds as a contiguous float32 device tensor of n values
    (numpy arrays and host tensors are copied to the device)."""
    if prior is None:
        return None
    t = prior if isinstance(prior, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(prior, dtype=np.float32))
    t = t.to(device="cuda", dtype=torch.float32).contiguous()
    if t.numel() != n:
        raise ValueError("prior must hold %d values, got %d" % (n, t.numel()))
    return t


def _policy(policy="gg", alpha=4, theta=0.05, seed=1, influence="prefix", mask_update="replace",
            stop="fixed_iters", mlp=None, tau=0.0, rho=1.0, fallback_k=0, audit=False, trace=None, label_eps=1e-3,
            alpha0=None, theta0=None, vstatus="none", eps=0.0):
    """alpha0 / theta0 (either one given): decoupled first-superstep parameters,
    the other defaulting to alpha / theta. vstatus ("none", "abs", "rel") and
    eps: GG-VStatus of PR/PPR."""
    dec = alpha0 is not None or theta0 is not None
    return Policy(POLICY[policy], alpha, theta, seed, INFLUENCE[influence], MASK[mask_update], STOP[stop],
                  None if mlp is None else mlp.handle.value, float(tau), float(rho), int(fallback_k), int(bool(audit)),
                  None if trace is None else trace.handle.value, float(label_eps), int(dec),
                  int(alpha if alpha0 is None else alpha0), float(theta if theta0 is None else theta0),
                  VSTATUS[vstatus], float(eps))


VSTATUS = {"none": 0, "abs": 1, "rel": 2}
POLICY_KW = ("mlp", "tau", "rho", "fallback_k", "audit", "trace", "label_eps", "alpha0", "theta0", "vstatus", "eps")


class Graph:
    """A graph loaded into the library (gg_graph_load_csr).

    rowptr/col/weight may be numpy arrays (copied to the device) or int32
    device tensors (borrowed: this object keeps them alive).
    """

    def __init__(self, n, rowptr, col, weight=None, stream=None, validate=True, m=None):
        self._keep = (rowptr, col, weight)
        dev = isinstance(rowptr, torch.Tensor) and rowptr.is_cuda
        if dev:
            for t in (rowptr, col) + ((weight,) if weight is not None else ()):
                if t.dtype != torch.int32 or not t.is_contiguous():
                    raise TypeError("device CSR arrays must be contiguous int32 tensors")
        else:
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
            col = np.ascontiguousarray(col, dtype=np.int32)
            weight = None if weight is None else np.ascontiguousarray(weight, dtype=np.int32)
            self._keep = (rowptr, col, weight)
        self.n = int(n)
        self.m = int(col.shape[0]) if m is None else int(m)
        flags = (CSR_DEVICE_PTRS if dev else 0) | (0 if validate else CSR_SKIP_VALIDATE)
        desc = CsrDesc(self.n, self.m, _ptr(rowptr), _ptr(col), _ptr(weight), flags)
        h = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        _check(lib().gg_graph_load_csr(ctypes.byref(desc), self._stream, ctypes.byref(h)))
        self._h = h
        _live.add(self)
        self.weighted = weight is not None

    @classmethod
    def from_host(cls, g, device=True, stream=None, validate=True):
        """Load a graphgen.Graph-like object (n, rowptr, col, weight)."""
        m = int(g.rowptr[-1])
        if device:
            dev = torch.device("cuda")

            def up(a):
                # at least one element, so that an empty array still has a non-null address
                t = torch.zeros(max(m, 1), dtype=torch.int32, device=dev)
                if m:
                    t[:m].copy_(torch.from_numpy(np.ascontiguousarray(a[:m], dtype=np.int32)))
                return t

            rp = torch.from_numpy(np.ascontiguousarray(g.rowptr, dtype=np.int32)).to(dev)
            cl = up(g.col)
            w = None if g.weight is None else up(g.weight)
            torch.cuda.synchronize()
            return cls(g.n, rp, cl, w, stream=stream, validate=validate, m=m)
        return cls(g.n, g.rowptr, g.col, g.weight, stream=stream, validate=validate)

    def close(self):
        if getattr(self, "_h", None):
            lib().gg_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream):
        self._stream = _stream_handle(stream)
        _check(lib().gg_graph_set_stream(self._h, self._stream))

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().gg_graph_get_tuning(self._h, ctypes.byref(t)))
        return {k: int(getattr(t, k)) for k in TUNING_FIELDS}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        for k, v in kw.items():
            if k not in cur:
                raise KeyError(k)
            if v is not None:
                cur[k] = int(v)
        t = Tuning(*[cur[k] for k in TUNING_FIELDS])
        _check(lib().gg_graph_set_tuning(self._h, ctypes.byref(t)))

    def set_wait_limit(self, polls):
        """gg_graph_set_wait_limit: polls before a superstep's bounded wait gives up."""
        _check(lib().gg_graph_set_wait_limit(self._h, int(polls)))

    def set_parts(self, part_start, part_sources=None):
        """gg_graph_set_parts: part_start has n_parts + 1 entries (None or [] clears)."""
        if part_start is None or len(part_start) == 0:
            _check(lib().gg_graph_set_parts(self._h, 0, None, None))
            return
        ps = np.ascontiguousarray(part_start, dtype=np.int32)
        src = None if part_sources is None else np.ascontiguousarray(part_sources, dtype=np.int32)
        self._parts = (ps, src)
        _check(lib().gg_graph_set_parts(self._h, int(ps.shape[0]) - 1, ps.ctypes.data,
                                        None if src is None else src.ctypes.data))

    def set_capture(self, enable=True):
        """gg_graph_set_capture: capture and replay static whole-run schedules."""
        _check(lib().gg_graph_set_capture(self._h, 1 if enable else 0))

    def set_profiling(self, enable=True):
        _check(lib().gg_graph_set_profiling(self._h, 1 if enable else 0))

    def get_profile(self, kind, app) -> dict:
        p = KernelProfile()
        _check(lib().gg_graph_get_profile(self._h, PROFILE_KIND[kind], APP[app], ctypes.byref(p)))
        return {"launches": p.launches, "total_ms": p.total_ms, "alg_bytes": p.alg_bytes, "edges": p.edges}

    def _out(self, app, out):
        if out is None:
            out = torch.empty(self.n, dtype=_value_dtype(app), device="cuda")
        return out

    def exact_run(self, app, out=None, damping=0.85, iters=20, max_iters=1 << 20, source=0, dangling="uniform",
                  coupling=0.0, prior=None):
        """gg_exact_run: returns (values tensor on the device, Stats). BP takes
        coupling and prior (n float32 log-odds)."""
        out = self._out(app, out)
        pri = _prior_dev(prior, self.n)
        p = _app_params(app, damping, iters, max_iters, source, dangling, coupling=coupling, prior=pri)
        st = RunStats()
        _check(lib().gg_exact_run(self._h, ctypes.byref(p), out.data_ptr(), 0, ctypes.byref(st)))
        return out, _stats(st)

    def exact_run_noalloc(self, app, out, damping=0.85, iters=20, source=0, dangling="uniform"):
        """gg_exact_run_noalloc into a caller-allocated device tensor `out`;
        enqueues on the graph's stream without waiting. Returns (out, Stats)."""
        if not (out.is_cuda and out.dtype == _value_dtype(app) and out.is_contiguous() and out.numel() >= self.n):
            raise ValueError("out must be a contiguous device tensor of %d %s values" % (self.n, _value_dtype(app)))
        p = _app_params(app, damping, iters, 1, source, dangling)
        st = RunStats()
        _check(lib().gg_exact_run_noalloc(self._h, ctypes.byref(p), out.data_ptr(), ctypes.byref(st)))
        return out, _stats(st)

    def approx_run(self, app, sample_ratio, policy="gg", out=None, alpha=4, theta=0.05, seed=1,
                   influence="prefix", mask_update="replace", stop="fixed_iters", damping=0.85, iters=20,
                   max_iters=1 << 20, source=0, dangling="uniform", pr_degree="full", coupling=0.0, prior=None,
                   **learned):
        """gg_approx_run: returns (values tensor on the device, Stats). Learned-policy
        and trace arguments: mlp, tau, rho, fallback_k, audit, trace, label_eps;
        decoupled first superstep: alpha0, theta0; vertex status: vstatus, eps;
        pr_degree "full" or "active"; BP: coupling, prior."""
        bad = set(learned) - set(POLICY_KW)
        if bad:
            raise TypeError("unknown arguments %s" % sorted(bad))
        out = self._out(app, out)
        pri = _prior_dev(prior, self.n)
        p = _app_params(app, damping, iters, max_iters, source, dangling, pr_degree, coupling, pri)
        pol = _policy(policy, alpha, theta, seed, influence, mask_update, stop, **learned)
        st = RunStats()
        _check(lib().gg_approx_run(self._h, ctypes.byref(p), float(sample_ratio), ctypes.byref(pol),
                                   out.data_ptr(), 0, ctypes.byref(st)))
        return out, _stats(st)

    def batch_run(self, app, sources, sample_ratio=1.0, policy="exact", out=None, seed=1, damping=0.85, iters=20,
                  max_iters=1 << 20, dangling="uniform", alpha=0, pr_degree="full"):
        """gg_batch_run: returns (values [n, Q] on the device, Stats). pr_degree
        "active": PPR's approximate iterations divide by the sample's out-degree."""
        src = np.ascontiguousarray(sources, dtype=np.int32)
        q = int(src.shape[0])
        if out is None:
            out = torch.empty((self.n, q), dtype=_value_dtype(app), device="cuda")
        p = _app_params(app, damping, iters, max_iters, 0, dangling, pr_degree)
        pol = _policy(policy, alpha, 0.0, seed)
        st = RunStats()
        _check(lib().gg_batch_run(self._h, ctypes.byref(p), q, src.ctypes.data, float(sample_ratio),
                                  ctypes.byref(pol), out.data_ptr(), 0, ctypes.byref(st)))
        return out, _stats(st)

    def autotune(self, app, sample_ratio=1.0, policy="exact", sources=None, reps=2, damping=0.85, iters=20,
                 max_iters=1 << 20, source=0, dangling="uniform", coupling=0.0, prior=None, **pol):
        """gg_graph_autotune: times the workload (a single run, or a batch over
        `sources`) under candidate tunings and keeps the fastest on the graph.
        Returns (tuning dict, median ms of the chosen tuning)."""
        pri = _prior_dev(prior, self.n)
        p = _app_params(app, damping, iters, max_iters, source, dangling, coupling=coupling, prior=pri)
        pc = _policy(policy, **pol)
        src = None if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
        t = Tuning()
        ms = ctypes.c_double(0.0)
        _check(lib().gg_graph_autotune(self._h, ctypes.byref(p), float(sample_ratio), ctypes.byref(pc),
                                       0 if src is None else int(src.shape[0]),
                                       None if src is None else src.ctypes.data, int(reps), ctypes.byref(t),
                                       ctypes.byref(ms)))
        return {k: int(getattr(t, k)) for k in TUNING_FIELDS}, float(ms.value)

    def begin(self, app, sample_ratio=1.0, policy="exact", **kw) -> "Run":
        return Run(self, app, sample_ratio, policy, **kw)

    def update(self, del_src=(), del_dst=(), ins_src=(), ins_dst=(), ins_weight=None):
        """gg_graph_update: delete every arc matching (del_src[i], del_dst[i]),
        then insert ins_src[j] -> ins_dst[j] (weight ins_weight[j] on weighted
        graphs). No run may be active."""
        b, keep = _batch(del_src, del_dst, ins_src, ins_dst, ins_weight)
        _check(lib().gg_graph_update(self._h, ctypes.byref(b)))
        self.m = self._csr_m()
        self._keep = None  # the graph owns its CSR now

    def _csr_m(self) -> int:
        return int(lib().gg_graph_num_arcs(self._h))

    def csr(self, weights=False):
        """Host copies (rowptr, col, weight or None) of the graph's in-CSR."""
        rp = np.empty(self.n + 1, dtype=np.int32)
        _check(lib().gg_graph_get_csr(self._h, rp.ctypes.data, None, None))
        m = int(rp[-1])
        col = np.empty(max(m, 1), dtype=np.int32)
        w = np.empty(max(m, 1), dtype=np.int32) if weights else None
        _check(lib().gg_graph_get_csr(self._h, rp.ctypes.data, col.ctypes.data, None if w is None else w.ctypes.data))
        return rp, col[:m], None if w is None else w[:m]


class Run:
    """Step API (gg_run_begin / gg_run_step / gg_run_values / gg_run_mask /
    gg_run_export_state / gg_run_import_state / gg_run_end)."""

    def __init__(self, graph: Graph, app, sample_ratio=1.0, policy="exact", alpha=4, theta=0.05, seed=1,
                 influence="prefix", mask_update="replace", stop="fixed_iters", damping=0.85, iters=20,
                 max_iters=1 << 20, source=0, dangling="uniform", pr_degree="full", coupling=0.0, prior=None,
                 **learned):
        bad = set(learned) - set(POLICY_KW)
        if bad:
            raise TypeError("unknown arguments %s" % sorted(bad))
        self.graph = graph
        self.app = app
        self._keep = (learned.get("mlp"), learned.get("trace"))  # the run reads them until it ends
        pri = _prior_dev(prior, graph.n)  # copied by gg_run_begin
        p = _app_params(app, damping, iters, max_iters, source, dangling, pr_degree, coupling, pri)
        pol = _policy(policy, alpha, theta, seed, influence, mask_update, stop, **learned)
        h = ctypes.c_void_p()
        _check(lib().gg_run_begin(graph.handle, ctypes.byref(p), float(sample_ratio), ctypes.byref(pol),
                                  ctypes.byref(h)))
        self._h = h
        _live.add(self)

    def step(self) -> Optional[dict]:
        info = StepInfo()
        r = _check(lib().gg_run_step(self._h, ctypes.byref(info)))
        if r == 0:
            return None
        return {"iter": info.iter, "accurate": bool(info.accurate), "superstep": bool(info.superstep),
                "edges": info.edges, "changed": info.changed, "active_edges": info.active_edges,
                "edges_processed": info.edges_processed, "sparse": bool(info.sparse),
                "kind": STEP_KIND[info.kind], "selected": info.selected}

    def vstatus(self) -> np.ndarray:
        """gg_run_vstatus: uint8 [n], 1 for the vertices active after the last iteration."""
        out = np.zeros(max(self.graph.n, 1), dtype=np.uint8)
        _check(lib().gg_run_vstatus(self._h, out.ctypes.data))
        return out[: self.graph.n]

    def features(self) -> np.ndarray:
        """[n, 8] bfloat16 bits of the last correction step's features."""
        out = np.zeros((max(self.graph.n, 1), MLP_IN), dtype=np.uint16)
        _check(lib().gg_run_features(self._h, out.ctypes.data))
        return out[: self.graph.n]

    def selection(self):
        """(selected uint8 [n], logits float32 [n]) of the last LEARNED correction step."""
        sel = np.zeros(max(self.graph.n, 1), dtype=np.uint8)
        lg = np.zeros(max(self.graph.n, 1), dtype=np.float32)
        _check(lib().gg_run_selection(self._h, sel.ctypes.data, lg.ctypes.data))
        return sel[: self.graph.n], lg[: self.graph.n]

    def labels(self) -> np.ndarray:
        """Drift labels uint8 [n] of the last traced or audited full superstep."""
        out = np.zeros(max(self.graph.n, 1), dtype=np.uint8)
        _check(lib().gg_run_labels(self._h, out.ctypes.data))
        return out[: self.graph.n]

    def values(self, host=True):
        dt = {"pr": np.float32, "ppr": np.float32, "bp": np.float32, "sssp": np.uint32, "cc": np.int32}[self.app]
        if host:
            out = np.empty(max(self.graph.n, 1), dtype=dt)
            _check(lib().gg_run_values(self._h, out.ctypes.data, OUT_HOST))
            return out[: self.graph.n]
        out = torch.empty(self.graph.n, dtype=_value_dtype(self.app), device="cuda")
        _check(lib().gg_run_values(self._h, out.data_ptr(), 0))
        return out

    def update(self, del_src=(), del_dst=(), ins_src=(), ins_dst=(), ins_weight=None, more_iters=0):
        """gg_run_update: apply an update batch to the run's graph and continue
        for more_iters further iterations. Returns the reset vertices (uint8[n])."""
        b, keep = _batch(del_src, del_dst, ins_src, ins_dst, ins_weight)
        reset = np.empty(max(self.graph.n, 1), dtype=np.uint8)  # every byte written on success
        _check(lib().gg_run_update(self._h, ctypes.byref(b), int(more_iters), reset.ctypes.data))
        self.graph.m = self.graph._csr_m()
        self.graph._keep = None
        return reset[: self.graph.n]

    def mask_bits(self) -> np.ndarray:
        nw = (self.graph.m + 31) // 32
        out = np.zeros(max(nw, 1), dtype=np.uint32)
        _check(lib().gg_run_mask(self._h, out.ctypes.data))
        return out[:nw]

    def mask(self) -> np.ndarray:
        """Per-edge flags as uint8[m]."""
        bits = self.mask_bits()
        b = np.unpackbits(bits.view(np.uint8), bitorder="little")
        return b[: self.graph.m].astype(np.uint8)

    def stats(self) -> Stats:
        st = RunStats()
        _check(lib().gg_run_stats_get(self._h, ctypes.byref(st)))
        return _stats(st)

    def export_state(self) -> np.ndarray:
        """gg_run_export_state: the run's state after its last iteration, as host bytes."""
        size = ctypes.c_int64()
        _check(lib().gg_run_state_size(self._h, ctypes.byref(size)))
        out = np.zeros(size.value, dtype=np.uint8)
        _check(lib().gg_run_export_state(self._h, out.ctypes.data, size.value))
        return out

    def import_state(self, state) -> None:
        """gg_run_import_state: continue from a state that export_state returned."""
        buf = np.ascontiguousarray(state, dtype=np.uint8)
        _check(lib().gg_run_import_state(self._h, buf.ctypes.data, buf.size))

    def close(self):
        if getattr(self, "_h", None):
            # a graph that was freed first has already ended its run
            if getattr(self.graph, "_h", None):
                lib().gg_run_end(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Mlp:
    """The learned-correction network (gg_mlp_*). Calls run on `stream`
    (default: torch's current stream at creation)."""

    def __init__(self, seed=1, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().gg_mlp_create(_stream_handle(stream), int(seed), ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def set_weights(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError("expected %d parameters" % MLP_PARAMS)
        _check(lib().gg_mlp_set_weights(self.handle, p.ctypes.data))

    def get_weights(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().gg_mlp_get_weights(self.handle, p.ctypes.data))
        return p

    def forward(self, feat: torch.Tensor) -> torch.Tensor:
        """Logits of feat ([n, 8] bfloat16 bits as int16/uint16 on the device)."""
        assert feat.is_cuda and feat.is_contiguous() and feat.shape[-1] == MLP_IN and feat.element_size() == 2
        n = feat.shape[0]
        out = torch.empty(max(n, 1), dtype=torch.float32, device=feat.device)
        _check(lib().gg_mlp_forward(self.handle, feat.data_ptr(), n, out.data_ptr()))
        return out[:n]

    def loss_grad(self, feat: torch.Tensor, label: torch.Tensor, pos_weight=1.0) -> torch.Tensor:
        """[MLP_PARAMS + 1] float32: the gradient of the mean loss, then the loss sum."""
        assert feat.is_cuda and feat.is_contiguous() and feat.element_size() == 2
        assert label.is_cuda and label.dtype == torch.float32 and label.is_contiguous()
        out = torch.empty(MLP_PARAMS + 1, dtype=torch.float32, device=feat.device)
        _check(lib().gg_mlp_loss_grad(self.handle, feat.data_ptr(), label.data_ptr(), feat.shape[0],
                                      float(pos_weight), out.data_ptr()))
        return out

    def adam_step(self, grad: torch.Tensor, lr: float):
        assert grad.is_cuda and grad.dtype == torch.float32 and grad.numel() >= MLP_PARAMS
        _check(lib().gg_mlp_adam_step(self.handle, grad.data_ptr(), float(lr)))

    def train(self, trace: "Trace", epochs=5, batch=4096, lr=1e-3, pos_weight=1.0, seed=1) -> np.ndarray:
        """gg_mlp_train: returns the mean loss of every epoch."""
        losses = np.zeros(epochs, dtype=np.float32)
        _check(lib().gg_mlp_train(self.handle, trace.handle, int(epochs), int(batch), float(lr), float(pos_weight),
                                  int(seed), losses.ctypes.data))
        return losses

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().gg_mlp_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trace:
    """A device-resident trace of (features, drift label) samples (gg_trace_*)."""

    def __init__(self, capacity):
        h = ctypes.c_void_p()
        _check(lib().gg_trace_create(int(capacity), ctypes.byref(h)))
        self.handle = h
        _live.add(self)

    def clear(self):
        _check(lib().gg_trace_clear(self.handle))

    def info(self) -> dict:
        size, pos, dropped = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gg_trace_info(self.handle, ctypes.byref(size), ctypes.byref(pos), ctypes.byref(dropped)))
        return {"size": size.value, "positives": pos.value, "dropped": dropped.value}

    def export(self, first=0, count=None):
        """(features uint16 [count, 8], labels float32 [count]) on the host."""
        if count is None:
            count = self.info()["size"] - first
        f = np.zeros((max(count, 1), MLP_IN), dtype=np.uint16)
        y = np.zeros(max(count, 1), dtype=np.float32)
        _check(lib().gg_trace_export(self.handle, int(first), int(count), f.ctypes.data, y.ctypes.data))
        return f[:count], y[:count]

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().gg_trace_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
