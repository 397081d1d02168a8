"""Seeded synthetic graph inputs shared by the oracle tests and the GPU tests.

This package produces inputs only (edge lists, canonical in-CSR arrays,
weights, query sources). It contains none of the graph method's arithmetic.

Canonical in-CSR: row u lists the sources v of the arcs v -> u, sorted by
(v, generation index); self-loops are removed and duplicate arcs are kept.
Edge id e is the position in this CSR.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

# Graph500 R-MAT quadrant probabilities.
RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = False) -> str:
    """Compile the generator library (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


@functools.lru_cache(maxsize=None)
def _lib():
    build()
    lib = ctypes.CDLL(_LIB)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    lib.graphgen_draw.restype = ctypes.c_uint64
    lib.graphgen_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
    lib.graphgen_draws.restype = None
    lib.graphgen_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p]
    lib.graphgen_rmat_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.graphgen_er_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
    lib.graphgen_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.graphgen_apply_permutation.argtypes = [ctypes.c_int64, i32p, i32p, i32p]
    lib.graphgen_weights.argtypes = [ctypes.c_int64, ctypes.c_uint64, i32p]
    lib.graphgen_build_in_csr.restype = ctypes.c_int64
    lib.graphgen_build_in_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, ctypes.c_int32,
                                          i32p, i32p, ctypes.c_void_p]
    lib.graphgen_outdeg.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p]
    lib.graphgen_pick_sources.restype = ctypes.c_int32
    lib.graphgen_pick_sources.argtypes = [ctypes.c_int32, i32p, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_int64, i32p]
    return lib


@dataclass
class Graph:
    """A canonical in-CSR graph held in host memory."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[m], source of each in-edge
    weight: Optional[np.ndarray] = None  # int32[m] in [1, 255], or None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.rowptr[-1])

    def outdeg(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n).astype(np.int32)

    def indeg(self) -> np.ndarray:
        return np.diff(self.rowptr).astype(np.int32)

    def dst(self) -> np.ndarray:
        """Destination of every edge (row index), int32[m]."""
        return np.repeat(np.arange(self.n, dtype=np.int32), self.indeg())


def from_edges(n: int, src, dst, weight=None, symmetrize: bool = False, name: str = "") -> Graph:
    """Canonical in-CSR of an explicit arc list (generation index = list position)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = int(src.shape[0])
    if m and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    cap = 2 * m if symmetrize else m
    rowptr = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(max(cap, 1), dtype=np.int32)
    gen = np.zeros(max(cap, 1), dtype=np.int64)
    got = _lib().graphgen_build_in_csr(n, m, src, dst, int(symmetrize), rowptr, col,
                                       gen.ctypes.data_as(ctypes.c_void_p))
    if got < 0:
        raise MemoryError("graphgen_build_in_csr failed (%d)" % got)
    col = col[:got].copy()
    w = None
    if weight is not None:
        weight = np.asarray(weight, dtype=np.int32)
        g = gen[:got]
        w = weight[np.where(g >= m, g - m, g)].astype(np.int32)
    return Graph(n=n, rowptr=rowptr, col=col, weight=w, name=name)


def _cache_dir() -> Optional[str]:
    d = os.environ.get("GG_GRAPH_CACHE", "/tmp/gg_graph_cache")
    if d in ("", "0", "off"):
        return None
    os.makedirs(d, exist_ok=True)
    return d


def _cached(key: str, make):
    d = _cache_dir()
    paths = None
    if d is not None:
        paths = {k: os.path.join(d, "%s.%s.npy" % (key, k)) for k in ("meta", "rowptr", "col", "weight")}
        if all(os.path.exists(paths[k]) for k in ("meta", "rowptr", "col")):
            meta = np.load(paths["meta"])
            w = np.load(paths["weight"]) if os.path.exists(paths["weight"]) else None
            return Graph(n=int(meta[0]), rowptr=np.load(paths["rowptr"]), col=np.load(paths["col"]),
                         weight=w, name=key)
    g = make()
    g.name = key
    if paths is not None and g.m >= (1 << 20):
        for k, arr in (("rowptr", g.rowptr), ("col", g.col), ("weight", g.weight)):
            if arr is not None:
                tmp = paths[k] + ".tmp%d.npy" % os.getpid()
                np.save(tmp, arr)
                os.replace(tmp, paths[k])
        tmp = paths["meta"] + ".tmp%d.npy" % os.getpid()
        np.save(tmp, np.array([g.n], dtype=np.int64))
        os.replace(tmp, paths["meta"])
    return g


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, abc=RMAT_ABC, permute: bool = True,
         weights: bool = False, symmetrize: bool = False) -> Graph:
    """Seeded R-MAT graph, n = 2^scale, edge_factor * n generated pairs.

    Vertex ids are relabelled by a seeded permutation (stream seed + 0x1000);
    weights (if requested) are drawn per generated pair (stream seed + 0x2000).
    """
    key = "rmat_s%d_ef%d_seed%d_%s%s%s%s" % (scale, edge_factor, seed, "_".join("%g" % x for x in abc),
                                             "_perm" if permute else "", "_w" if weights else "",
                                             "_sym" if symmetrize else "")

    def make():
        n = 1 << scale
        m = edge_factor * n
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        lib = _lib()
        lib.graphgen_rmat_edges(scale, m, abc[0], abc[1], abc[2], seed, src, dst)
        if permute:
            perm = np.empty(n, dtype=np.int32)
            lib.graphgen_permutation(n, seed + 0x1000, perm)
            lib.graphgen_apply_permutation(m, perm, src, dst)
        w = None
        if weights:
            w = np.empty(m, dtype=np.int32)
            lib.graphgen_weights(m, seed + 0x2000, w)
        return from_edges(n, src, dst, w, symmetrize=symmetrize)

    return _cached(key, make)


def erdos_renyi(n: int, avg_degree: int = 16, seed: int = 4, weights: bool = False,
                symmetrize: bool = False) -> Graph:
    """Seeded Erdos-Renyi-style multigraph: avg_degree * n pairs with uniform endpoints."""
    key = "er_n%d_d%d_seed%d%s%s" % (n, avg_degree, seed, "_w" if weights else "",
                                     "_sym" if symmetrize else "")

    def make():
        m = avg_degree * n
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        lib = _lib()
        lib.graphgen_er_edges(n, m, seed, src, dst)
        w = None
        if weights:
            w = np.empty(m, dtype=np.int32)
            lib.graphgen_weights(m, seed + 0x2000, w)
        return from_edges(n, src, dst, w, symmetrize=symmetrize)

    return _cached(key, make)


def pick_sources(g: Graph, count: int, seed: int) -> np.ndarray:
    """`count` query sources with out-degree > 0, drawn with replacement (stream seed + 0x3000)."""
    out = np.empty(max(count, 1), dtype=np.int32)
    od = np.ascontiguousarray(g.outdeg(), dtype=np.int32)
    got = _lib().graphgen_pick_sources(g.n, od, count, seed + 0x3000, 1 << 40, out)
    if got < count:
        raise ValueError("graph has no vertex with out-degree > 0")
    return out[:count].copy()


def bp_prior(n: int, seed: int) -> np.ndarray:
    """Prior log-odds of a belief-propagation workload, float32 [n]: every
    vertex carries evidence of its own strength, a probability p of state 1
    uniform in [0.05, 0.95] (log-odds within +-2.944, no two vertices tied).
    Uses the generator's own counter-based draws: vertex u takes
    draw(seed, u, 0)."""
    u = np.empty(max(n, 1), dtype=np.uint64)
    _lib().graphgen_draws(seed, 0, n, u.ctypes.data)
    a = (u[:n] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    p = 0.05 + 0.9 * a
    return (np.log(p) - np.log1p(-p)).astype(np.float32)


def draw(seed: int, k: int, l: int = 0) -> int:
    return int(_lib().graphgen_draw(seed, k, l))


# --- small structured graphs -------------------------------------------------

def dumbbell(k: int = 5, weight: int = 1) -> Graph:
    """Two k-cliques joined by one undirected bridge (both arcs) between vertex k-1 and k."""
    src, dst = [], []
    for base in (0, k):
        for i in range(k):
            for j in range(k):
                if i != j:
                    src.append(base + i)
                    dst.append(base + j)
    src += [k - 1, k]
    dst += [k, k - 1]
    w = [weight] * len(src)
    return from_edges(2 * k, src, dst, w, name="dumbbell%d" % k)


def directed_cycle(n: int) -> Graph:
    src = list(range(n))
    dst = [(i + 1) % n for i in range(n)]
    return from_edges(n, src, dst, [1] * n, name="cycle%d" % n)


def star(n: int, inward: bool = True) -> Graph:
    """Star on n vertices with centre 0; arcs leaf -> centre if inward else centre -> leaf."""
    leaves = list(range(1, n))
    src, dst = (leaves, [0] * (n - 1)) if inward else ([0] * (n - 1), leaves)
    return from_edges(n, src, dst, [1] * (n - 1), name="star%d" % n)


def complete(n: int) -> Graph:
    src = [i for i in range(n) for j in range(n) if i != j]
    dst = [j for i in range(n) for j in range(n) if i != j]
    return from_edges(n, src, dst, [1] * len(src), name="complete%d" % n)


def random_small(n: int, m: int, seed: int, max_weight: int = 255) -> Graph:
    """Small random multigraph (with possible self-loops, which the CSR drops)."""
    rng = np.random.Generator(np.random.Philox(seed))
    src = rng.integers(0, n, size=m).astype(np.int32)
    dst = rng.integers(0, n, size=m).astype(np.int32)
    w = rng.integers(1, max_weight + 1, size=m).astype(np.int32)
    return from_edges(n, src, dst, w, name="rand_n%d_m%d_s%d" % (n, m, seed))


def tiny_family():
    """Small graphs covering cycles, stars, cliques, DAGs, dangling-heavy and random cases."""
    gs = [directed_cycle(5), directed_cycle(1 + 7), star(6, True), star(6, False), complete(5),
          dumbbell(4)]
    # DAG: i -> j for i < j with a sparse pattern
    src = [i for i in range(8) for j in range(i + 1, 8) if (i * 7 + j) % 3 == 0]
    dst = [j for i in range(8) for j in range(i + 1, 8) if (i * 7 + j) % 3 == 0]
    gs.append(from_edges(8, src, dst, [1 + (k % 9) for k in range(len(src))], name="dag8"))
    # dangling-heavy: most vertices have no out-edges
    gs.append(from_edges(10, [0, 1, 2, 3, 0, 1], [4, 5, 6, 7, 8, 9], [3, 1, 4, 1, 5, 9], name="dangling10"))
    # graph with isolated vertices
    gs.append(from_edges(7, [0, 1, 2], [1, 2, 0], [2, 2, 2], name="isolated7"))
    for s in range(8):
        gs.append(random_small(6 + s, 4 * (6 + s), seed=100 + s))
    return gs


def union(graphs, name: str = "union"):
    """Block-diagonal union of graphs: graph p's vertices are offset by the
    vertex count of graphs 0..p-1. Returns (Graph, part_start) with
    part_start[p] = first vertex of graph p and part_start[-1] = n."""
    part_start = [0]
    rowptrs, cols, weights = [], [], []
    e_off = 0
    for g in graphs:
        rowptrs.append(np.asarray(g.rowptr[:-1], dtype=np.int64) + e_off)
        cols.append(np.asarray(g.col, dtype=np.int64) + part_start[-1])
        weights.append(g.weight)
        e_off += g.m
        part_start.append(part_start[-1] + g.n)
    n = part_start[-1]
    rowptr = np.concatenate(rowptrs + [np.array([e_off])]).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    w = None
    if all(x is not None for x in weights):
        w = np.concatenate(weights).astype(np.int32)
    return Graph(n=n, rowptr=rowptr, col=col, weight=w, name=name), np.array(part_start, dtype=np.int32)


def part(g: Graph, part_start, p: int) -> Graph:
    """Graph p of a block-diagonal union, with local vertex ids."""
    v0, v1 = int(part_start[p]), int(part_start[p + 1])
    e0, e1 = int(g.rowptr[v0]), int(g.rowptr[v1])
    rowptr = (g.rowptr[v0:v1 + 1] - e0).astype(np.int32)
    col = (g.col[e0:e1] - v0).astype(np.int32)
    w = None if g.weight is None else g.weight[e0:e1].copy()
    return Graph(n=v1 - v0, rowptr=rowptr, col=col, weight=w, name="%s[%d]" % (g.name, p))


def rmat_family(count: int, scale_range=(10, 18), ef_range=(8, 32), seed0: int = 100, weights: bool = True,
                symmetrize: bool = False):
    """`count` independent R-MAT graphs with scale ~ U{scale_range} (log-uniform
    vertex counts) and edge factor ~ U{ef_range}; graph g uses seed seed0 + g."""
    out = []
    for k in range(count):
        sc = scale_range[0] + int(draw(seed0 + k, 0, 0) % (scale_range[1] - scale_range[0] + 1))
        ef = ef_range[0] + int(draw(seed0 + k, 0, 1) % (ef_range[1] - ef_range[0] + 1))
        out.append(rmat(sc, ef, seed=seed0 + k, weights=weights, symmetrize=symmetrize))
    return out
