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

PR, SSSP, CC, PPR = 0, 1, 2, 3
EXACT, SP, SMS, GG = 0, 1, 2, 3
FIXED_ITERS, FIXED_POINT = 0, 1
INFL_PREFIX, INFL_TOTAL = 0, 1
MASK_REPLACE, MASK_UNION = 0, 1
DANGLING_UNIFORM, DANGLING_NONE = 0, 1
INF = 0xFFFFFFFF

APP_NAMES = {"pr": PR, "sssp": SSSP, "cc": CC, "ppr": PPR}
POLICY_NAMES = {"exact": EXACT, "sp": SP, "sms": SMS, "gg": GG}


def build(force: bool = False) -> str:
    """Compile the oracle: plain single-threaded C at -O2."""
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
                ("max_iters", ctypes.c_int32), ("source", ctypes.c_int32), ("dangling", ctypes.c_int32)]


class _Pol(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("alpha", ctypes.c_int32), ("theta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64), ("influence", ctypes.c_int32),
                ("mask_update", ctypes.c_int32), ("stop", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("accurate", ctypes.c_int32), ("superstep", ctypes.c_int32),
                ("edges", ctypes.c_int64), ("changed", ctypes.c_int64), ("active_edges", ctypes.c_int64)]


@functools.lru_cache(maxsize=None)
def _lib():
    build()
    lib = ctypes.CDLL(_LIB)
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
    for f in ("ggo_get_values", "ggo_get_mask", "ggo_get_influence"):
        getattr(lib, f).argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.ggo_end.argtypes = [ctypes.c_void_p]
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
                 influence=INFL_PREFIX, mask_update=MASK_REPLACE, stop=FIXED_ITERS):
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
        ap = _App(self.app, damping, iters, max_iters, source, dangling)
        po = _Pol(kind, alpha, theta, sigma, seed, influence, mask_update, stop)
        self._h = self._lib.ggo_begin(ctypes.byref(csr), ctypes.byref(ap), ctypes.byref(po))
        if not self._h:
            raise ValueError("oracle: " + self._lib.ggo_last_error().decode())

    def step(self) -> Optional[StepInfo]:
        info = _Info()
        if not self._lib.ggo_step(self._h, ctypes.byref(info)):
            return None
        return StepInfo(info.iter, bool(info.accurate), bool(info.superstep), info.edges, info.changed,
                        info.active_edges)

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
        dt = {PR: np.float64, PPR: np.float64, SSSP: np.uint32, CC: np.int32}[self.app]
        out = np.empty(self.n, dtype=dt)
        self._lib.ggo_get_values(self._h, out.ctypes.data)
        return out

    def mask(self) -> np.ndarray:
        out = np.empty(max(self.m, 1), dtype=np.uint8)
        self._lib.ggo_get_mask(self._h, out.ctypes.data)
        return out[: self.m]

    def influence(self) -> np.ndarray:
        out = np.empty(max(self.m, 1), dtype=np.float64)
        self._lib.ggo_get_influence(self._h, out.ctypes.data)
        return out[: self.m]

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
