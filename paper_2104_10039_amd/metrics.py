"""Error metrics of approximate results against accurate-mode results
[Sec. 4.2], computed on the host.

- Top-K error (PageRank): fraction of the approximate top-k vertices that are
  not in the accurate top-k. Ranking is by value, descending, ties broken by
  the lower vertex id.
- Stretch error (SSSP): per vertex reachable in the accurate run (source
  excluded), (approximate - accurate) / accurate, capped at 1; a vertex the
  approximate run leaves unreached counts 1. The mean over those vertices.
- Relative error (CC): fraction of vertices whose approximate component label
  differs from the accurate one.
- Accuracy = (1 - error) * 100.
"""
from __future__ import annotations

import numpy as np

INF = 0xFFFFFFFF


def top_k(values, k: int) -> np.ndarray:
    """Ids of the k largest values, ties broken by the lower id, in rank
    order. Only the candidates at or above the k-th largest value are
    sorted."""
    v = np.asarray(values, dtype=np.float64)
    k = min(k, v.shape[0])
    if k <= 0:
        return np.zeros(0, dtype=np.int64)
    kth = np.partition(v, v.shape[0] - k)[v.shape[0] - k]
    cand = np.nonzero(v >= kth)[0]
    order = np.lexsort((cand, -v[cand]))
    return cand[order[:k]]


def topk_error(approx, exact, k: int = 1000) -> float:
    a = top_k(approx, k)
    e = top_k(exact, k)
    if a.size == 0:
        return 0.0
    return float(np.setdiff1d(a, e, assume_unique=True).size) / float(a.size)


def stretch_error(approx, exact, source: int) -> float:
    a = np.asarray(approx).astype(np.uint32).astype(np.float64)
    e = np.asarray(exact).astype(np.uint32).astype(np.float64)
    sel = (e != INF)
    sel[source] = False
    if not sel.any():
        return 0.0
    a, e = a[sel], e[sel]
    err = np.where(a == INF, 1.0, np.minimum((a - e) / np.maximum(e, 1.0), 1.0))
    return float(err.mean())


def label_mismatch(approx, exact) -> float:
    a = np.asarray(approx)
    e = np.asarray(exact)
    return float((a != e).mean()) if a.size else 0.0


def accuracy(error: float) -> float:
    return (1.0 - error) * 100.0
