"""Host-side error metrics [Sec. 4.2] against their plain definitions."""
import numpy as np

from paper_2104_10039_amd import metrics


def test_top_k_matches_full_sort_with_ties():
    rng = np.random.default_rng(3)
    for n, k in ((1, 1), (10, 3), (1000, 1000), (5000, 100), (20000, 1000)):
        v = rng.integers(0, 50, size=n).astype(np.float64)  # many ties
        ref = np.lexsort((np.arange(n), -v))[:k]
        assert np.array_equal(metrics.top_k(v, k), ref)
    assert metrics.top_k(np.zeros(0), 5).size == 0


def test_topk_error_and_accuracy():
    e = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    a = np.array([5.0, 1.0, 3.0, 2.0, 4.0])  # top-2 {0, 4} against {0, 1}
    assert metrics.topk_error(a, e, 2) == 0.5
    assert metrics.accuracy(metrics.topk_error(e, e, 3)) == 100.0


def test_stretch_and_labels():
    inf = metrics.INF
    exact = np.array([0, 10, 20, inf], dtype=np.uint32)
    approx = np.array([0, 15, inf, inf], dtype=np.uint32)
    # vertex 1: (15 - 10) / 10 = 0.5; vertex 2 unreached: 1; vertex 3 not reachable: excluded
    assert metrics.stretch_error(approx, exact, 0) == 0.75
    assert metrics.label_mismatch(np.array([0, 0, 2]), np.array([0, 1, 2])) == 1.0 / 3.0
