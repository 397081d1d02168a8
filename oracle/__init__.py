"""Python access to the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library. The GPU library never
imports it.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
# A prebuilt oracle library to load instead (the mutation tests point this at
# copies of the oracle with one planted mistake); build() leaves it alone.
_LIB_OVERRIDE = os.environ.get("GGO_ORACLE_LIB")

PR, SSSP, CC, PPR, BP = 0, 1, 2, 3, 4
EXACT, SP, SMS, GG, LEARNED = 0, 1, 2, 3, 4
KIND_APPROX, KIND_ACCURATE, KIND_FULL, KIND_PARTIAL = 0, 1, 2, 3
MLP_IN, MLP_HIDDEN = 8, 64
MLP_PARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + 2 * MLP_HIDDEN + 1
# offsets of the parameter vector: W1 [8][64], b1, W2 [64][64], b2, w3, b3
P_W1 = 0
P_B1 = P_W1 + MLP_IN * MLP_HIDDEN
P_W2 = P_B1 + MLP_HIDDEN
P_B2 = P_W2 + MLP_HIDDEN * MLP_HIDDEN
P_W3 = P_B2 + MLP_HIDDEN
P_B3 = P_W3 + MLP_HIDDEN
FIXED_ITERS, FIXED_POINT = 0, 1
INFL_PREFIX, INFL_TOTAL, INFL_PUSH = 0, 1, 2
MASK_REPLACE, MASK_UNION = 0, 1
DANGLING_UNIFORM, DANGLING_NONE = 0, 1
DEGREE_FULL, DEGREE_ACTIVE = 0, 1
VSTATUS_NONE, VSTATUS_ABS, VSTATUS_REL = 0, 1, 2
INF = 0xFFFFFFFF

APP_NAMES = {"pr": PR, "sssp": SSSP, "cc": CC, "ppr": PPR, "bp": BP}
POLICY_NAMES = {"exact": EXACT, "sp": SP, "sms": SMS, "gg": GG, "learned": LEARNED}


def build(force: bool = False) -> str:
    """Compile the oracle: plain single-threaded C at -O2."""
    if _LIB_OVERRIDE:
        return _LIB_OVERRIDE
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class _App(ctypes.Structure):
    _fields_ = [("app", ctypes.c_int32), ("damping", ctypes.c_double), ("iters", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("source", ctypes.c_int32), ("dangling", ctypes.c_int32),
                ("pr_degree", ctypes.c_int32), ("coupling", ctypes.c_double), ("prior", ctypes.c_void_p)]


class _Pol(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("alpha", ctypes.c_int32), ("theta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64), ("influence", ctypes.c_int32),
                ("mask_update", ctypes.c_int32), ("stop", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("tau", ctypes.c_double), ("rho", ctypes.c_double), ("fallback_k", ctypes.c_int32),
                ("trace", ctypes.c_int32), ("label_eps", ctypes.c_double), ("decoupled", ctypes.c_int32),
                ("alpha0", ctypes.c_int32), ("theta0", ctypes.c_double), ("vstatus", ctypes.c_int32),
                ("eps", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("accurate", ctypes.c_int32), ("superstep", ctypes.c_int32),
                ("edges", ctypes.c_int64), ("changed", ctypes.c_int64), ("active_edges", ctypes.c_int64),
                ("kind", ctypes.c_int32), ("selected", ctypes.c_int64)]


@functools.lru_cache(maxsize=None)
def _lib():
    lib = ctypes.CDLL(build())
    lib.ggo_philox4x64_10.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
    lib.ggo_sample_draw.restype = ctypes.c_uint32
    lib.ggo_sample_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64]
    lib.ggo_keep_threshold.restype = ctypes.c_uint64
    lib.ggo_keep_threshold.argtypes = [ctypes.c_double]
    lib.ggo_begin.restype = ctypes.c_void_p
    lib.ggo_begin.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_App), ctypes.POINTER(_Pol)]
    lib.ggo_step.restype = ctypes.c_int
    lib.ggo_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Info)]
    lib.ggo_done.restype = ctypes.c_int
    lib.ggo_done.argtypes = [ctypes.c_void_p]
    lib.ggo_iterations.restype = ctypes.c_int32
    lib.ggo_iterations.argtypes = [ctypes.c_void_p]
    lib.ggo_edges_total.restype = ctypes.c_int64
    lib.ggo_edges_total.argtypes = [ctypes.c_void_p]
    for f in ("ggo_get_values", "ggo_get_mask", "ggo_get_influence", "ggo_set_mask", "ggo_get_vactive",
              "ggo_set_vactive"):
        getattr(lib, f).argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_end.argtypes = [ctypes.c_void_p]
    lib.ggo_get_features.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_get_selection.restype = ctypes.c_int
    lib.ggo_get_selection.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_get_labels.restype = ctypes.c_int
    lib.ggo_get_labels.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_bf16_bits.restype = ctypes.c_uint16
    lib.ggo_bf16_bits.argtypes = [ctypes.c_float]
    lib.ggo_bf16_array.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    lib.ggo_bf16_value.restype = ctypes.c_float
    lib.ggo_bf16_value.argtypes = [ctypes.c_uint16]
    lib.ggo_run_update.restype = ctypes.c_int
    lib.ggo_run_update.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Csr), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32]
    lib.ggo_get_reset.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_bp_message.restype = ctypes.c_double
    lib.ggo_bp_message.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.ggo_lg_feature.restype = ctypes.c_float
    lib.ggo_lg_feature.argtypes = [ctypes.c_int64]
    lib.ggo_delta_feature.restype = ctypes.c_float
    lib.ggo_delta_feature.argtypes = [ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32]
    lib.ggo_mlp_forward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    lib.ggo_mlp_loss_grad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_adam_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.c_double, ctypes.c_int64]
    lib.ggo_last_error.restype = ctypes.c_char_p
    return lib


def philox4x64_10(counter, key):
    c = (ctypes.c_uint64 * 4)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in counter])
    k = (ctypes.c_uint64 * 2)(*[int(x) & 0xFFFFFFFFFFFFFFFF for x in key])
    o = (ctypes.c_uint64 * 4)()
    _lib().ggo_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def sample_draw(seed: int, epoch: int, e: int) -> int:
    return int(_lib().ggo_sample_draw(seed, epoch, e))


def keep_threshold(sigma: float) -> int:
    return int(_lib().ggo_keep_threshold(sigma))


@dataclass
class StepInfo:
    iter: int
    accurate: bool
    superstep: bool
    edges: int
    changed: int
    active_edges: int
    kind: int = KIND_APPROX
    selected: int = -1


@dataclass
class Result:
    values: np.ndarray
    iterations: int
    edges: int
    steps: List[StepInfo] = field(default_factory=list)
    mask: Optional[np.ndarray] = None


class Run:
    """A step-by-step oracle run (begin / step / values / mask / end)."""

    def __init__(self, g, app, policy="exact", sigma=1.0, alpha=4, theta=0.05, seed=1,
                 damping=0.85, iters=20, max_iters=100000, source=0, dangling=DANGLING_UNIFORM,
                 influence=INFL_PREFIX, mask_update=MASK_REPLACE, stop=FIXED_ITERS, mlp=None, tau=0.0,
                 rho=1.0, fallback_k=0, trace=False, label_eps=1e-3, pr_degree=DEGREE_FULL, alpha0=None,
                 theta0=None, vstatus=VSTATUS_NONE, eps=0.0, coupling=0.0, prior=None):
        self._lib = _lib()
        self.app = APP_NAMES[app] if isinstance(app, str) else int(app)
        kind = POLICY_NAMES[policy] if isinstance(policy, str) else int(policy)
        self.n = int(g.n)
        self.m = int(g.rowptr[-1])
        self._rowptr = np.ascontiguousarray(g.rowptr, dtype=np.int32)
        self._col = np.ascontiguousarray(g.col, dtype=np.int32)
        self._w = None if g.weight is None else np.ascontiguousarray(g.weight, dtype=np.int32)
        csr = _Csr(self.n, self.m, self._rowptr.ctypes.data, self._col.ctypes.data,
                   None if self._w is None else self._w.ctypes.data)
        # BP: prior log-odds (binary64, one per vertex) and edge coupling
        self._prior = None if prior is None else np.ascontiguousarray(prior, dtype=np.float64)
        if self._prior is not None and self._prior.size != self.n:
            raise ValueError("prior needs %d entries" % self.n)
        ap = _App(self.app, damping, iters, max_iters, source, dangling, pr_degree, coupling,
                  None if self._prior is None or self.n == 0 else self._prior.ctypes.data)
        self._mlp = None if mlp is None else np.ascontiguousarray(mlp, dtype=np.float64)
        if self._mlp is not None and self._mlp.size != MLP_PARAMS:
            raise ValueError("mlp needs %d parameters" % MLP_PARAMS)
        po = _Pol(kind, alpha, theta, sigma, seed, influence, mask_update, stop,
                  None if self._mlp is None else self._mlp.ctypes.data, tau, rho, fallback_k, int(bool(trace)),
                  label_eps, int(alpha0 is not None or theta0 is not None),
                  alpha if alpha0 is None else alpha0, theta if theta0 is None else theta0, vstatus, eps)
        self._h = self._lib.ggo_begin(ctypes.byref(csr), ctypes.byref(ap), ctypes.byref(po))
        if not self._h:
            raise ValueError("oracle: " + self._lib.ggo_last_error().decode())

    def step(self) -> Optional[StepInfo]:
        info = _Info()
        if not self._lib.ggo_step(self._h, ctypes.byref(info)):
            return None
        return StepInfo(info.iter, bool(info.accurate), bool(info.superstep), info.edges, info.changed,
                        info.active_edges, info.kind, info.selected)

    @property
    def done(self) -> bool:
        return bool(self._lib.ggo_done(self._h))

    @property
    def iterations(self) -> int:
        return int(self._lib.ggo_iterations(self._h))

    @property
    def edges_total(self) -> int:
        return int(self._lib.ggo_edges_total(self._h))

    def values(self) -> np.ndarray:
        dt = {PR: np.float64, PPR: np.float64, BP: np.float64, SSSP: np.uint32, CC: np.int32}[self.app]
        out = np.empty(self.n, dtype=dt)
        self._lib.ggo_get_values(self._h, out.ctypes.data)
        return out

    def mask(self) -> np.ndarray:
        out = np.empty(max(self.m, 1), dtype=np.uint8)
        self._lib.ggo_get_mask(self._h, out.ctypes.data)
        return out[: self.m]

    def update(self, upd: "Update", more_iters: int = 0):
        """Continue this run on the graph after an update batch (ggo_run_update)."""
        if upd.graph.n != self.n:
            raise ValueError("the vertex set of an update is fixed")
        g = upd.graph
        rp = np.ascontiguousarray(g.rowptr, dtype=np.int32)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        w = None if g.weight is None else np.ascontiguousarray(g.weight, dtype=np.int32)
        oon = np.ascontiguousarray(upd.old_of_new, dtype=np.int64)
        dele = np.ascontiguousarray(upd.deleted_old, dtype=np.uint8)
        m = int(rp[-1])
        csr = _Csr(self.n, m, rp.ctypes.data, col.ctypes.data, None if w is None else w.ctypes.data)
        if self._lib.ggo_run_update(self._h, ctypes.byref(csr), oon.ctypes.data if m else None,
                                    dele.ctypes.data if self.m else None, int(more_iters)) != 0:
            raise ValueError("oracle: " + self._lib.ggo_last_error().decode())
        # the run reads the new arrays until it ends
        self._rowptr, self._col, self._w = rp, col, w
        self.m = m

    def reset_vertices(self) -> np.ndarray:
        """Vertices whose value the last update reset (one byte per vertex)."""
        out = np.empty(max(self.n, 1), dtype=np.uint8)
        self._lib.ggo_get_reset(self._h, out.ctypes.data)
        return out[: self.n]

    def set_mask(self, mask):
        """Adopt another side's edge flags (one value per edge, nonzero = active)."""
        a = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
        if a.size != self.m:
            raise ValueError("mask needs %d entries" % self.m)
        self._lib.ggo_set_mask(self._h, a.ctypes.data if self.m else None)

    def vactive(self) -> np.ndarray:
        out = np.empty(max(self.n, 1), dtype=np.uint8)
        self._lib.ggo_get_vactive(self._h, out.ctypes.data)
        return out[: self.n]

    def set_vactive(self, act):
        a = np.ascontiguousarray(np.asarray(act) != 0, dtype=np.uint8)
        if a.size != self.n:
            raise ValueError("vertex status needs %d entries" % self.n)
        self._lib.ggo_set_vactive(self._h, a.ctypes.data if self.n else None)

    def influence(self) -> np.ndarray:
        out = np.empty(max(self.m, 1), dtype=np.float64)
        self._lib.ggo_get_influence(self._h, out.ctypes.data)
        return out[: self.m]

    def features(self) -> np.ndarray:
        """[n, 8] bfloat16 bits of the features of the last correction or traced step."""
        out = np.zeros((max(self.n, 1), MLP_IN), dtype=np.uint16)
        self._lib.ggo_get_features(self._h, out.ctypes.data)
        return out[: self.n]

    def selection(self):
        """(selected uint8 [n], logits float64 [n]) of this step, or None."""
        sel = np.zeros(max(self.n, 1), dtype=np.uint8)
        lg = np.zeros(max(self.n, 1), dtype=np.float64)
        if not self._lib.ggo_get_selection(self._h, sel.ctypes.data, lg.ctypes.data):
            return None
        return sel[: self.n], lg[: self.n]

    def labels(self):
        """Drift labels uint8 [n] of this step (traced full superstep), or None."""
        out = np.zeros(max(self.n, 1), dtype=np.uint8)
        if not self._lib.ggo_get_labels(self._h, out.ctypes.data):
            return None
        return out[: self.n]

    def close(self):
        if self._h:
            self._lib.ggo_end(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run_to_end(self, keep_steps=True) -> Result:
        steps = []
        while True:
            s = self.step()
            if s is None:
                break
            if keep_steps:
                steps.append(s)
        return Result(values=self.values(), iterations=self.iterations, edges=self.edges_total, steps=steps,
                      mask=self.mask())


def run(g, app, policy="exact", **kw) -> Result:
    r = Run(g, app, policy, **kw)
    try:
        return r.run_to_end()
    finally:
        r.close()


# ---------------------------------------------------------------------------
# bfloat16 and the correction MLP
# ---------------------------------------------------------------------------

def bf16_bits(x) -> int:
    return int(_lib().ggo_bf16_bits(float(x)))


def bf16_array(x) -> np.ndarray:
    """bfloat16 bits of a float32 array (round to nearest even)."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(a.shape, dtype=np.uint16)
    _lib().ggo_bf16_array(a.ctypes.data, out.ctypes.data, a.size)
    return out


def bf16_value(b) -> float:
    return float(_lib().ggo_bf16_value(int(b)))


def lg_feature(y) -> float:
    return float(_lib().ggo_lg_feature(int(y)))


def delta_feature(app, now, before) -> float:
    a = APP_NAMES[app] if isinstance(app, str) else int(app)
    return float(_lib().ggo_delta_feature(a, int(now) & 0xFFFFFFFF, int(before) & 0xFFFFFFFF))


def mlp_forward(params, feat, rounding=True) -> np.ndarray:
    """Logits of the samples in feat ([n, 8] bfloat16 bits)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.uint16).reshape(-1, MLP_IN)
    out = np.zeros(max(len(f), 1), dtype=np.float64)
    _lib().ggo_mlp_forward(p.ctypes.data, f.ctypes.data, len(f), int(bool(rounding)), out.ctypes.data)
    return out[: len(f)]


def mlp_loss_grad(params, feat, label, pos_weight=1.0, rounding=True):
    """(mean loss, gradient [MLP_PARAMS]) of the weighted BCE-with-logits loss."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.uint16).reshape(-1, MLP_IN)
    y = np.ascontiguousarray(label, dtype=np.float32)
    g = np.zeros(MLP_PARAMS, dtype=np.float64)
    loss = ctypes.c_double()
    _lib().ggo_mlp_loss_grad(p.ctypes.data, f.ctypes.data, y.ctypes.data, len(f), float(pos_weight),
                             int(bool(rounding)), g.ctypes.data, ctypes.byref(loss))
    return loss.value, g


def adam_step(params, m, v, grad, lr, t):
    """In-place Adam step on float64 arrays."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float64)
    _lib().ggo_adam_step(params.ctypes.data, m.ctypes.data, v.ctypes.data, g.ctypes.data, params.size, float(lr),
                         int(t))


def bp_message(L, coupling):
    """The oracle's BP message log-ratio of a sender with log-odds L."""
    return float(_lib().ggo_bp_message(float(L), float(coupling)))


# ---------------------------------------------------------------------------
# Dynamic graphs: the graph after an update batch (plain definition)
# ---------------------------------------------------------------------------

@dataclass
class UpdatedCsr:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    weight: Optional[np.ndarray] = None

    @property
    def m(self) -> int:
        return int(self.rowptr[-1])


@dataclass
class Update:
    graph: UpdatedCsr
    old_of_new: np.ndarray   # int64[m_new]: the old edge each new edge continues, -1 if inserted
    deleted_old: np.ndarray  # uint8[m_old]: 1 for every old edge the batch removed


def apply_update(g, del_src, del_dst, ins_src, ins_dst, ins_weight=None) -> Update:
    """The in-CSR after an update batch. Deletions remove every arc s -> d of
    the graph that matches a listed pair (s, d); insertions then add one arc
    per listed triple. Each row stays sorted by source; among arcs with the
    same source, the surviving ones come first in their old order, then the
    inserted ones in batch order. The vertex set is fixed. The rows of g
    must be sorted by source (the canonical in-CSR)."""
    n = int(g.n)
    rowptr = np.asarray(g.rowptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    m = int(rowptr[-1])
    dst = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    if m > 1 and np.any((dst[1:] == dst[:-1]) & (col[1:] < col[:-1])):
        raise ValueError("a row is not sorted by source")
    del_src = np.asarray(del_src, dtype=np.int64)
    del_dst = np.asarray(del_dst, dtype=np.int64)
    ins_src = np.asarray(ins_src, dtype=np.int64)
    ins_dst = np.asarray(ins_dst, dtype=np.int64)
    for a in (del_src, del_dst, ins_src, ins_dst):
        if a.size and (a.min() < 0 or a.max() >= n):
            raise ValueError("vertex id out of range")
    if ins_src.size != ins_dst.size or del_src.size != del_dst.size:
        raise ValueError("source and destination lists differ in length")
    if g.weight is None and ins_weight is not None:
        raise ValueError("weights inserted into a graph without weights")
    if g.weight is not None:
        if ins_weight is None:
            ins_weight = np.zeros(0, dtype=np.int64) if ins_src.size == 0 else None
        if ins_weight is None or np.asarray(ins_weight).size != ins_src.size:
            raise ValueError("a weighted graph needs one weight per inserted arc")
        if np.asarray(ins_weight).size and (np.min(ins_weight) < 0 or np.max(ins_weight) > 255):
            raise ValueError("weight outside [0, 255]")
    deleted = np.isin(col * n + dst, del_src * n + del_dst)
    keep = np.nonzero(~deleted)[0]
    k_ins = ins_src.size
    # every arc of the new graph: (destination, source, group 0 = old / 1 = inserted, order within group)
    d_all = np.concatenate([dst[keep], ins_dst])
    s_all = np.concatenate([col[keep], ins_src])
    grp = np.concatenate([np.zeros(keep.size, dtype=np.int64), np.ones(k_ins, dtype=np.int64)])
    within = np.concatenate([keep, np.arange(k_ins, dtype=np.int64)])
    order = np.lexsort((within, grp, s_all, d_all))
    new_rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(new_rowptr, d_all + 1, 1)
    new_rowptr = np.cumsum(new_rowptr)
    old_of_new = np.where(grp[order] == 0, within[order], -1)
    weight = None
    if g.weight is not None:
        w_all = np.concatenate([np.asarray(g.weight, dtype=np.int64)[keep],
                                np.asarray(ins_weight, dtype=np.int64).reshape(-1)])
        weight = w_all[order].astype(np.int32)
    out = UpdatedCsr(n, new_rowptr.astype(np.int32), s_all[order].astype(np.int32), weight)
    return Update(out, old_of_new.astype(np.int64), deleted.astype(np.uint8))
