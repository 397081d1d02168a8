"""Pins of the CPU oracle against things other than itself.

Library routines (numpy's Philox, scipy's Dijkstra and connected components,
numpy linear solves), closed forms, special cases in which the method reduces
to a textbook algorithm, invariants, and hand-worked examples in
tests/golden/. None of these tests needs a GPU.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# Counter-based sampling draw (Philox4x64-10 of Salmon et al. 2011)
# --------------------------------------------------------------------------

def numpy_philox_block(counter, key):
    """Philox4x64-10(counter, key) via numpy, whose generator pre-increments the counter."""
    cint = sum(int(c) << (64 * i) for i, c in enumerate(counter))
    prev = (cint - 1) % (1 << 256)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([(prev >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((12345, 3, 0, 0), (99, 0)),
    ((M64, M64, M64, M64), (M64, M64)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89), (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(counter, key):
    assert oracle.philox4x64_10(counter, key) == numpy_philox_block(counter, key)


def test_sample_draw_layout():
    seed, epoch = 0xDEADBEEF, 0
    for e in list(range(0, 40)) + [1 << 20, (1 << 31) + 5]:
        words = numpy_philox_block((e >> 3, epoch, 0, 0), (seed, 0))
        j = e & 7
        w = words[j >> 1]
        want = (w >> 32) if (j & 1) else (w & 0xFFFFFFFF)
        assert oracle.sample_draw(seed, epoch, e) == want


def test_keep_threshold_endpoints():
    assert oracle.keep_threshold(0.0) == 0
    assert oracle.keep_threshold(1.0) == 1 << 32
    assert oracle.keep_threshold(0.5) == 1 << 31


@pytest.mark.parametrize("sigma", [0.0, 0.1, 0.3, 0.5, 0.7, 0.9, 1.0])
def test_initial_mask_is_bernoulli_sigma(sigma):
    """The initial flags equal an independent numpy computation of the draws,
    and the kept fraction lies within 5 binomial standard deviations."""
    g = gg.rmat(12, 16, seed=7)
    r = oracle.Run(g, "pr", "sp", sigma=sigma, seed=11, iters=1)
    mask = r.mask()
    m = g.m
    # independent draws for a sample of edges
    rng = np.random.default_rng(3)
    idx = rng.integers(0, m, size=200)
    thr = int(np.floor(sigma * 2 ** 32 + 0.5))
    for e in idx:
        words = numpy_philox_block((int(e) >> 3, 0, 0, 0), (11, 0))
        j = int(e) & 7
        w = words[j >> 1]
        d = (w >> 32) if (j & 1) else (w & 0xFFFFFFFF)
        assert mask[e] == (1 if d < thr else 0)
    kept = int(mask.sum())
    if sigma in (0.0, 1.0):
        assert kept == int(sigma * m)
    else:
        sd = np.sqrt(m * sigma * (1 - sigma))
        assert abs(kept - sigma * m) < 5 * sd


# --------------------------------------------------------------------------
# Exact iterations against textbook routines
# --------------------------------------------------------------------------

def _adj(g, weights=False, keep=None):
    """Sparse adjacency A[v, u] for arcs v -> u; parallel arcs collapse to their
    minimum weight (a shortest path uses the lightest of them)."""
    src, dst = g.col, g.dst()
    w = g.weight.astype(np.float64) if weights else np.ones(g.m)
    if keep is not None:
        keep = keep.astype(bool)
        src, dst, w = src[keep], dst[keep], w[keep]
    key = src.astype(np.int64) * g.n + dst
    order = np.lexsort((w, key))
    key, w = key[order], w[order]
    first = np.ones(len(key), dtype=bool)
    first[1:] = key[1:] != key[:-1]
    key, w = key[first], w[first]
    # zero weights would vanish from a sparse matrix; they do not occur in these graphs
    assert np.all(w > 0)
    return sp.csr_matrix((w, (key // g.n, key % g.n)), shape=(g.n, g.n))


def pr_linear_solve(g, d=0.85, dangling=True, source=None):
    """Fixed point of PageRank (or personalized PageRank) by a dense linear solve."""
    n = g.n
    outdeg = g.outdeg().astype(np.float64)
    A = np.zeros((n, n))
    np.add.at(A, (g.dst(), g.col), 1.0)  # A[u, v] = multiplicity of v -> u
    W = A / np.where(outdeg > 0, outdeg, 1.0)[None, :]
    dang = (outdeg == 0).astype(np.float64) if dangling else np.zeros(n)
    if source is None:
        M = np.eye(n) - d * (W + np.outer(np.ones(n) / n, dang))
        b = np.full(n, (1 - d) / n)
    else:
        es = np.zeros(n)
        es[source] = 1.0
        M = np.eye(n) - d * (W + np.outer(es, dang))
        b = (1 - d) * es
    return np.linalg.solve(M, b)


def pr_dense_power(g, iters, d=0.85):
    """T steps of the dense power iteration with uniform dangling redistribution."""
    n = g.n
    outdeg = g.outdeg().astype(np.float64)
    A = np.zeros((n, n))
    np.add.at(A, (g.dst(), g.col), 1.0)
    W = A / np.where(outdeg > 0, outdeg, 1.0)[None, :]
    G = d * (W + np.outer(np.ones(n) / n, (outdeg == 0).astype(np.float64)))
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = (1 - d) / n + G @ x
    return x


@pytest.mark.parametrize("gi", range(len(gg.tiny_family())))
def test_pr_exact_vs_dense_power_iteration(gi):
    g = gg.tiny_family()[gi]
    got = oracle.run(g, "pr", iters=20).values
    want = pr_dense_power(g, 20)
    assert np.max(np.abs(got - want)) <= 1e-12
    assert abs(got.sum() - 1.0) <= 1e-12  # mass is conserved with uniform dangling


def test_pr_exact_converges_to_linear_solve():
    for g in [gg.rmat(8, 8, seed=3), gg.random_small(30, 90, seed=5), gg.dumbbell(5)]:
        got = oracle.run(g, "pr", iters=300).values
        want = pr_linear_solve(g)
        assert np.max(np.abs(got - want)) <= 1e-12


def test_ppr_exact_converges_to_linear_solve():
    g = gg.random_small(25, 80, seed=9)
    s = int(gg.pick_sources(g, 1, 9)[0])
    got = oracle.run(g, "ppr", iters=300, source=s).values
    want = pr_linear_solve(g, source=s)
    assert np.max(np.abs(got - want)) <= 1e-12
    assert abs(got.sum() - 1.0) <= 1e-12


def test_pr_closed_forms():
    # directed cycle and a complete graph: every vertex has rank 1/N
    for g in [gg.directed_cycle(7), gg.complete(6)]:
        got = oracle.run(g, "pr", iters=20).values
        assert np.max(np.abs(got - 1.0 / g.n)) <= 1e-15
    # in-star: leaves have no in-edges, the centre collects all leaves; no dangling leaves
    n, d = 6, 0.85
    g = gg.star(n, inward=True)
    x = oracle.run(g, "pr", iters=1).values
    # one iteration from 1/N: the centre is dangling (mass 1/N spread), leaves get (1-d)/N + d*(1/N)/N
    leaf = (1 - d) / n + d * (1.0 / n) / n
    centre = (1 - d) / n + d * ((n - 1) * (1.0 / n) + (1.0 / n) / n)
    assert abs(x[1] - leaf) < 1e-16 and abs(x[0] - centre) < 1e-15


def _sssp_graphs():
    gs = [g for g in gg.tiny_family()]
    gs.append(gg.rmat(10, 8, seed=21, weights=True))
    gs.append(gg.erdos_renyi(1 << 10, 4, seed=22, weights=True))
    return gs


@pytest.mark.parametrize("gi", range(len(_sssp_graphs())))
def test_sssp_exact_vs_dijkstra(gi):
    g = _sssp_graphs()[gi]
    srcs = gg.pick_sources(g, 2, 5 + gi)
    for s in srcs:
        r = oracle.run(g, "sssp", source=int(s))
        want = csg.dijkstra(_adj(g, weights=True), directed=True, indices=int(s))
        want_u = np.where(np.isinf(want), oracle.INF, want).astype(np.uint32)
        assert np.array_equal(r.values, want_u)
        # exact run stops after the first iteration that changes nothing
        assert r.steps[-1].changed == 0 and all(st.changed > 0 for st in r.steps[:-1])


def test_sssp_triangle_inequality_at_fixed_point():
    g = gg.rmat(11, 8, seed=31, weights=True)
    s = int(gg.pick_sources(g, 1, 31)[0])
    x = oracle.run(g, "sssp", source=s).values.astype(np.int64)
    dst = g.dst()
    fin = x[g.col] != oracle.INF
    assert np.all(x[dst][fin] <= x[g.col][fin] + g.weight[fin])


def _cc_graphs():
    gs = []
    for g in gg.tiny_family()[:6]:
        gs.append(g)
    gs.append(gg.rmat(10, 4, seed=41, symmetrize=True))
    gs.append(gg.erdos_renyi(1 << 10, 1, seed=42, symmetrize=True))
    return gs


def min_label_components(g):
    ncomp, lab = csg.connected_components(_adj(g), directed=True, connection="weak")
    mins = np.full(ncomp, g.n, dtype=np.int64)
    np.minimum.at(mins, lab, np.arange(g.n))
    return mins[lab].astype(np.int32)


@pytest.mark.parametrize("gi", range(len(_cc_graphs())))
def test_cc_exact_vs_union_find(gi):
    g = _cc_graphs()[gi]
    if not _is_symmetric(g):
        g = gg.from_edges(g.n, g.col, g.dst(), symmetrize=True)
    r = oracle.run(g, "cc")
    assert np.array_equal(r.values, min_label_components(g))


def _is_symmetric(g):
    A = _adj(g)
    return (A != A.T).nnz == 0


# --------------------------------------------------------------------------
# Special cases of the approximate schedule
# --------------------------------------------------------------------------

@pytest.mark.parametrize("app", ["pr", "sssp", "cc", "ppr"])
def test_alpha_zero_and_sigma_one_equal_exact(app):
    g = gg.rmat(10, 8, seed=51, weights=True, symmetrize=(app == "cc"))
    s = int(gg.pick_sources(g, 1, 51)[0])
    exact = oracle.run(g, app, "exact", source=s)
    kw = dict(source=s, iters=exact.iterations)
    # alpha = 0: every iteration is a superstep (accurate)
    a0 = oracle.run(g, app, "gg", sigma=0.3, alpha=0, theta=0.2, **kw)
    assert np.array_equal(a0.values, exact.values)
    # sigma = 1 with SP: every edge stays active
    s1 = oracle.run(g, app, "sp", sigma=1.0, **kw)
    assert np.array_equal(s1.values, exact.values)
    # SMS with alpha = 0 switches to accurate mode immediately
    sms = oracle.run(g, app, "sms", sigma=0.2, alpha=0, **kw)
    assert np.array_equal(sms.values, exact.values)


def test_pr_theta_zero_keeps_every_edge():
    """PR contributions are positive, so every influence is > 0 = theta."""
    g = gg.rmat(10, 8, seed=52)
    exact = oracle.run(g, "pr", "exact")
    r = oracle.run(g, "pr", "gg", sigma=1.0, alpha=1, theta=0.0)
    assert np.array_equal(r.values, exact.values)
    assert r.mask.all()


def _submatrix(g, mask, weights=False):
    return _adj(g, weights=weights, keep=mask)


@pytest.mark.parametrize("sigma", [0.2, 0.5, 0.8])
def test_sp_fixed_point_is_exact_on_sampled_subgraph_sssp(sigma):
    g = gg.rmat(10, 8, seed=61, weights=True)
    s = int(gg.pick_sources(g, 1, 61)[0])
    r = oracle.run(g, "sssp", "sp", sigma=sigma, seed=5, stop=oracle.FIXED_POINT, source=s)
    want = csg.dijkstra(_submatrix(g, r.mask, weights=True), directed=True, indices=s)
    assert np.array_equal(r.values, np.where(np.isinf(want), oracle.INF, want).astype(np.uint32))


@pytest.mark.parametrize("sigma", [0.2, 0.5, 0.8])
def test_sp_fixed_point_is_exact_on_sampled_subgraph_cc(sigma):
    """On a (possibly asymmetric) sampled arc set, label propagation converges
    to the minimum id among the vertices that reach u (u included)."""
    g = gg.rmat(8, 4, seed=62, symmetrize=True)
    r = oracle.run(g, "cc", "sp", sigma=sigma, seed=6, stop=oracle.FIXED_POINT)
    A = _submatrix(g, r.mask)
    reach = csg.shortest_path(A, directed=True, unweighted=True)  # reach[v, u] finite iff v reaches u
    want = np.array([min([v for v in range(g.n) if np.isfinite(reach[v, u])]) for u in range(g.n)])
    assert np.array_equal(r.values, want.astype(np.int32))


def test_sp_pr_fixed_point_linear_solve():
    """SP PageRank with full out-degrees is the linear iteration on the sampled
    arcs; its fixed point solves (I - d(W_s + 1 dang^T / N)) x = (1-d)/N."""
    g = gg.random_small(20, 70, seed=63)
    r = oracle.run(g, "pr", "sp", sigma=0.6, seed=7, iters=400)
    keep = r.mask.astype(bool)
    n, d = g.n, 0.85
    outdeg = g.outdeg().astype(np.float64)
    A = np.zeros((n, n))
    np.add.at(A, (g.dst()[keep], g.col[keep]), 1.0)
    W = A / np.where(outdeg > 0, outdeg, 1.0)[None, :]
    M = np.eye(n) - d * (W + np.outer(np.ones(n) / n, (outdeg == 0).astype(np.float64)))
    want = np.linalg.solve(M, np.full(n, (1 - d) / n))
    assert np.max(np.abs(r.values - want)) <= 1e-12


# --------------------------------------------------------------------------
# Hand-worked examples (tests/golden)
# --------------------------------------------------------------------------

def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_golden_pr_superstep():
    fx = _load("pr_superstep_4v.json")
    edges = fx["graph"]["edges"]
    g = gg.from_edges(fx["graph"]["n"], [e[0] for e in edges], [e[1] for e in edges])
    p = fx["params"]
    r = oracle.Run(g, "pr", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], iters=p["iters"],
                   damping=0.85)
    for it in range(1, p["iters"] + 1):
        st = r.step()
        want = np.array([float(Fraction(v)) for v in fx["expected"]["values_after"][str(it)]])
        assert np.max(np.abs(r.values() - want)) <= 1e-15, it
        if it == 2:
            assert st.superstep
            assert list(r.mask()) == fx["expected"]["mask_after_superstep_2"]
            want_infl = np.array([float(Fraction(v)) for v in fx["expected"]["influence_at_superstep_2"]])
            assert np.max(np.abs(r.influence() - want_infl)) <= 1e-7  # binary32 contributions


def _u32(v):
    return oracle.INF if v == "INF" else int(v)


def test_golden_sssp_superstep():
    fx = _load("sssp_superstep_4v.json")
    edges = fx["graph"]["edges"]
    g = gg.from_edges(fx["graph"]["n"], [e[0] for e in edges], [e[1] for e in edges], [e[2] for e in edges])
    p = fx["params"]
    r = oracle.Run(g, "sssp", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], iters=p["iters"],
                   source=p["source"])
    gathered = []
    for it in range(1, p["iters"] + 1):
        st = r.step()
        gathered.append(st.edges)
        assert list(r.values()) == [_u32(v) for v in fx["expected"]["values_after"][str(it)]], it
        if str(it) in fx["expected"]["mask_after"]:
            assert list(r.mask()) == fx["expected"]["mask_after"][str(it)], it
    assert gathered == fx["expected"]["edges_gathered"]
    assert r.done
    ex = oracle.run(g, "sssp", "exact", source=p["source"])
    assert list(ex.values) == fx["expected"]["exact_values"]
    assert ex.iterations == fx["expected"]["exact_iterations"]


def test_golden_cc_dumbbell():
    fx = _load("cc_dumbbell_gg.json")
    g = gg.dumbbell(fx["graph"]["dumbbell_k"])
    p = fx["params"]
    r = oracle.Run(g, "cc", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], stop=oracle.FIXED_POINT)
    dst = g.dst()
    for it in range(1, 5):
        r.step()
        if str(it) in fx["expected"]["values_after"]:
            assert list(r.values()) == fx["expected"]["values_after"][str(it)], it
        if it == 2:
            act = sorted((int(g.col[e]), int(dst[e])) for e in np.nonzero(r.mask())[0])
            assert act == sorted(tuple(a) for a in fx["expected"]["active_arcs_after_2"])
    res = r.run_to_end()
    assert list(res.values) == fx["expected"]["final"]
    assert res.iterations == fx["expected"]["iterations"]


def test_dumbbell_bridge_dropped_by_sampling_restored_by_superstep():
    """Sec. 2.4 / Fig. 1b: with a seed whose uniform sample drops both bridge
    arcs, SP leaves two components; GG's superstep restores one component."""
    g = gg.dumbbell(5)
    dst = g.dst()
    bridge = [e for e in range(g.m) if {int(g.col[e]), int(dst[e])} == {4, 5}]
    thr = 1 << 31
    seed = None
    for s in range(1, 500):
        draws = []
        for e in bridge:
            words = numpy_philox_block((e >> 3, 0, 0, 0), (s, 0))
            w = words[(e & 7) >> 1]
            draws.append((w >> 32) if (e & 1) else (w & 0xFFFFFFFF))
        if all(d >= thr for d in draws):
            seed = s
            break
    assert seed is not None
    sp_ = oracle.run(g, "cc", "sp", sigma=0.5, seed=seed, stop=oracle.FIXED_POINT)
    assert not any(sp_.mask[e] for e in bridge)
    assert len(set(sp_.values.tolist())) >= 2
    assert set(sp_.values[:5].tolist()).isdisjoint(set(sp_.values[5:].tolist()))
    gg_ = oracle.run(g, "cc", "gg", sigma=0.5, seed=seed, alpha=2, theta=0.5, stop=oracle.FIXED_POINT)
    assert np.all(gg_.values == 0)


# --------------------------------------------------------------------------
# Influence properties and invariants of the approximate runs
# --------------------------------------------------------------------------

def test_prefix_influence_first_edge_and_telescoping():
    g = gg.rmat(10, 8, seed=71)
    r = oracle.Run(g, "pr", "gg", sigma=0.5, alpha=1, theta=0.3, iters=2)
    r.step()
    r.step()  # superstep
    infl = r.influence()
    mask = r.mask()
    for u in range(g.n):
        b, e = g.rowptr[u], g.rowptr[u + 1]
        if e > b:
            assert infl[b] == 1.0 and mask[b] == 1  # the first edge of a row has influence 1
            # P_k = P_{k-1} / (1 - infl_k) telescopes back to P_1 = c_1 > 0
            for k in range(b + 1, e):
                assert 0.0 < infl[k] <= 1.0
    assert np.array_equal(mask, (infl > 0.3).astype(np.uint8))


def test_cc_argmin_edge_always_active_after_superstep():
    g = gg.rmat(9, 4, seed=72, symmetrize=True)
    r = oracle.Run(g, "cc", "gg", sigma=0.3, alpha=2, theta=0.5, stop=oracle.FIXED_POINT)
    lab_prev = r.values()
    while not r.done:
        st = r.step()
        if st.superstep:
            mask = r.mask()
            for u in range(g.n):
                b, e = g.rowptr[u], g.rowptr[u + 1]
                if e > b:
                    src_lab = lab_prev[g.col[b:e]]
                    k = int(np.argmin(src_lab))
                    assert mask[b + k] == 1
        lab_prev = r.values()


@pytest.mark.parametrize("policy,sigma", [("sp", 0.3), ("gg", 0.3), ("gg", 0.7), ("sms", 0.5)])
def test_sssp_approximate_invariants(policy, sigma):
    g = gg.rmat(10, 8, seed=81, weights=True)
    s = int(gg.pick_sources(g, 1, 81)[0])
    exact = oracle.run(g, "sssp", "exact", source=s).values.astype(np.int64)
    r = oracle.Run(g, "sssp", policy, sigma=sigma, alpha=2, theta=0.1, source=s, stop=oracle.FIXED_POINT)
    prev = r.values().astype(np.int64)
    while not r.done:
        r.step()
        cur = r.values().astype(np.int64)
        assert np.all(cur <= prev)  # monotone non-increasing
        fin = cur != oracle.INF
        assert np.all(cur[fin] >= exact[fin])  # never below the true distance
        prev = cur
    # each finite value is realised by an in-edge (a real path, by induction)
    dst = g.dst()
    fin = (prev != oracle.INF)
    for u in np.nonzero(fin)[0]:
        if u == s:
            assert prev[u] == 0
            continue
        b, e = g.rowptr[u], g.rowptr[u + 1]
        cand = prev[g.col[b:e]] + g.weight[b:e]
        assert np.any(cand == prev[u])
    if policy != "sp":  # fixed point of an accurate iteration: certified exact
        assert np.array_equal(prev, exact)


def test_cc_gg_fixed_point_is_exact():
    g = gg.rmat(10, 4, seed=82, symmetrize=True)
    exact = oracle.run(g, "cc", "exact").values
    for sigma in (0.1, 0.5):
        r = oracle.run(g, "cc", "gg", sigma=sigma, alpha=3, theta=0.5, stop=oracle.FIXED_POINT)
        assert np.array_equal(r.values, exact)
        assert np.all(r.values <= np.arange(g.n))


def test_periodic_schedule():
    g = gg.rmat(8, 4, seed=83)
    r = oracle.run(g, "pr", "gg", sigma=0.5, alpha=4, theta=0.05, iters=20)
    assert [s.iter for s in r.steps if s.accurate] == [5, 10, 15, 20]
    assert all(s.superstep == s.accurate for s in r.steps)
    r = oracle.run(g, "pr", "sms", sigma=0.5, alpha=4, iters=20)
    assert [s.iter for s in r.steps if s.accurate] == list(range(5, 21))
    assert not any(s.superstep for s in r.steps)
    r = oracle.run(g, "pr", "sp", sigma=0.5, iters=20)
    assert not any(s.accurate for s in r.steps)
    m = r.mask
    assert all(s.edges == int(m.sum()) for s in r.steps)


def test_mask_union_keeps_old_flags():
    g = gg.rmat(9, 8, seed=84)
    a = oracle.run(g, "pr", "gg", sigma=0.5, alpha=1, theta=0.3, iters=2)
    b = oracle.run(g, "pr", "gg", sigma=0.5, alpha=1, theta=0.3, iters=2, mask_update=oracle.MASK_UNION)
    init = oracle.Run(g, "pr", "sp", sigma=0.5, iters=1).mask()
    assert np.array_equal(b.mask, a.mask | init)


def test_invalid_arguments_rejected():
    g = gg.rmat(6, 4, seed=85, weights=True)
    with pytest.raises(ValueError):
        oracle.Run(g, "pr", "gg", sigma=1.5)
    with pytest.raises(ValueError):
        oracle.Run(g, "pr", "gg", theta=-1.0)
    with pytest.raises(ValueError):
        oracle.Run(g, "sssp", "exact", source=g.n)
    gnw = gg.rmat(6, 4, seed=85)
    with pytest.raises(ValueError):
        oracle.Run(gnw, "sssp", "exact", source=0)


# ---------------------------------------------------------------------------
# EStatus decisions on hand-built rows (values worked out by hand)
# ---------------------------------------------------------------------------

def _eid(g, s, d):
    """Edge id of the arc s -> d in the canonical in-CSR (first occurrence)."""
    row = g.col[g.rowptr[d]:g.rowptr[d + 1]]
    return int(g.rowptr[d] + int(np.nonzero(row == s)[0][0]))


def test_sssp_estatus_improvement_is_relative_to_the_old_minimum():
    """Row 3 sees candidates 100 (via 1) then 95 (via 2) at the superstep of
    iteration 2. The improvement (100 - 95) / 100 = 0.05 does not exceed
    theta = 0.05 (strict, compared as 5 * 2^16 = 327680 against
    round(0.05 * 2^16) * 100 = 327700), so the arc 2 -> 3 is deactivated; the
    first finite candidate is always active [Alg. 2, GG-EStatus; reading 10]."""
    g = gg.from_edges(4, [0, 0, 1, 2], [1, 2, 3, 3], [50, 45, 50, 50], name="sssp_rel")
    r = oracle.Run(g, "sssp", "gg", sigma=1.0, alpha=1, theta=0.05, seed=1, iters=2, source=0)
    r.step()
    r.step()
    mask = r.mask()
    assert mask[_eid(g, 1, 3)] == 1 and mask[_eid(g, 2, 3)] == 0
    assert list(r.values()) == [0, 50, 45, 95]
    r.close()


def test_sssp_unreached_source_keeps_its_flag():
    """Path 0 -> 1 -> 2 -> 3: at the superstep of iteration 2 vertex 2 is
    still unreached, so the arc 2 -> 3 cannot be assessed and keeps its flag
    (active, sigma = 1); the assessed arcs stay active as first finite
    candidates [Sec. 3.4; reading 11]."""
    g = gg.from_edges(4, [0, 1, 2], [1, 2, 3], [1, 1, 1], name="sssp_path")
    r = oracle.Run(g, "sssp", "gg", sigma=1.0, alpha=1, theta=0.05, seed=1, iters=2, source=0)
    r.step()
    r.step()
    assert list(r.mask()) == [1, 1, 1]
    r.close()


def test_estatus_is_strict_for_binary_cc_influence():
    """Triangle 0-1-2 (both directions), every iteration a superstep
    (alpha = 0), theta = 0: row 2 reads label 0 (via 0, influence 1) then
    label 1 (via 1, influence 0); 0 > 0 is false, so the arc 1 -> 2 is
    deactivated [Alg. 2, GG-EStatus: active iff influence > threshold]."""
    g = gg.from_edges(3, [0, 1, 0, 2, 1, 2], [1, 0, 2, 0, 2, 1], None, name="triangle")
    r = oracle.Run(g, "cc", "gg", sigma=1.0, alpha=0, theta=0.0, seed=1, iters=1)
    r.step()
    mask = r.mask()
    assert mask[_eid(g, 0, 2)] == 1 and mask[_eid(g, 1, 2)] == 0
    assert mask[_eid(g, 0, 1)] == 1 and mask[_eid(g, 2, 1)] == 0
    r.close()


# --------------------------------------------------------------------------
# Variants: dangling mass dropped, TOTAL influence, ACTIVE out-degree,
# decoupled first-superstep parameters, GG-VStatus, the replay hooks
# --------------------------------------------------------------------------

def test_pr_dangling_none_linear_solve():
    """Dropping the dangling mass (the literal Alg. 2 apply) is the linear
    iteration x = (1-d)/N + d W x, whose fixed point a dense solve gives; PPR
    likewise with the teleport to the source."""
    g = gg.random_small(24, 40, seed=62)
    assert np.sum(g.outdeg() == 0) >= 3, "the pin needs dangling vertices"
    r = oracle.run(g, "pr", "exact", iters=400, dangling=oracle.DANGLING_NONE)
    want = pr_linear_solve(g, dangling=False)
    assert np.max(np.abs(r.values - want)) <= 1e-12
    assert r.values.sum() < 1.0 - 1e-3  # mass leaks through the dangling vertices
    s = int(np.nonzero(g.outdeg() > 0)[0][0])
    r = oracle.run(g, "ppr", "exact", iters=400, source=s, dangling=oracle.DANGLING_NONE)
    assert np.max(np.abs(r.values - pr_linear_solve(g, dangling=False, source=s))) <= 1e-12


def _golden_graph(fx):
    edges = fx["graph"]["edges"]
    return gg.from_edges(fx["graph"]["n"], [e[0] for e in edges], [e[1] for e in edges])


def _fr(vals):
    return np.array([float(Fraction(v)) for v in vals])


def test_golden_pr_total_influence():
    fx = _load("pr_total_influence_4v.json")
    g, p = _golden_graph(fx), fx["params"]
    r = oracle.Run(g, "pr", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], iters=p["iters"],
                   influence=oracle.INFL_TOTAL)
    for it in range(1, p["iters"] + 1):
        st = r.step()
        assert np.max(np.abs(r.values() - _fr(fx["expected"]["values_after"][str(it)]))) <= 1e-15, it
        if it == 2:
            assert st.superstep
            assert list(r.mask()) == fx["expected"]["mask_after_superstep_2"]
            assert np.max(np.abs(r.influence() - _fr(fx["expected"]["influence_at_superstep_2"]))) <= 1e-7
    # PREFIX keeps every edge at this threshold: the two readings differ here
    q = oracle.run(g, "pr", "gg", sigma=1.0, alpha=1, theta=p["theta"], iters=2)
    assert list(q.mask) == [1] * 6


def test_golden_pr_active_degree():
    fx = _load("pr_active_degree_4v.json")
    g, p = _golden_graph(fx), fx["params"]
    r = oracle.Run(g, "pr", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], iters=p["iters"],
                   pr_degree=oracle.DEGREE_ACTIVE)
    for it in range(1, p["iters"] + 1):
        r.step()
        assert np.max(np.abs(r.values() - _fr(fx["expected"]["values_after"][str(it)]))) <= 1e-15, it
        if it == 2:
            assert list(r.mask()) == fx["expected"]["mask_after_superstep_2"]
    assert abs(r.values().sum() - 1.0) <= 1e-15


def test_active_degree_sp_is_pagerank_of_the_sampled_graph():
    """SP with the ACTIVE out-degree run to its fixed point is textbook
    PageRank (uniform dangling mass) of the materialised sampled subgraph,
    solved densely; with sigma = 1 it equals the full-degree run bit for bit."""
    g = gg.random_small(30, 110, seed=77)
    r = oracle.run(g, "pr", "sp", sigma=0.55, seed=5, iters=500, pr_degree=oracle.DEGREE_ACTIVE)
    keep = r.mask.astype(bool)
    sub = gg.from_edges(g.n, g.col[keep], g.dst()[keep])
    want = pr_linear_solve(sub)
    assert np.max(np.abs(r.values - want)) <= 1e-12
    assert abs(r.values.sum() - 1.0) <= 1e-12
    a = oracle.run(g, "pr", "gg", sigma=1.0, alpha=2, theta=0.0, iters=9, pr_degree=oracle.DEGREE_ACTIVE)
    b = oracle.run(g, "pr", "gg", sigma=1.0, alpha=2, theta=0.0, iters=9)
    assert np.array_equal(a.values, b.values)


def test_golden_pr_decoupled_parameters():
    fx = _load("pr_decoupled_4v.json")
    g, p = _golden_graph(fx), fx["params"]
    r = oracle.Run(g, "pr", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], alpha0=p["alpha0"],
                   theta0=p["theta0"], iters=p["iters"])
    supers = []
    for it in range(1, p["iters"] + 1):
        st = r.step()
        if st.superstep:
            supers.append(it)
        assert np.max(np.abs(r.values() - _fr(fx["expected"]["values_after"][str(it)]))) <= 1e-15, it
        if str(it) in fx["expected"]["mask_after"]:
            assert list(r.mask()) == fx["expected"]["mask_after"][str(it)], it
    assert supers == fx["expected"]["supersteps"]


@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_decoupled_with_equal_parameters_is_gg(app):
    """alpha0 = alpha and theta0 = theta reduce the decoupled schedule to GG's."""
    g = gg.rmat(8, 8, seed=21, weights=(app == "sssp"), symmetrize=(app == "cc"))
    kw = dict(sigma=0.4, alpha=3, theta=0.1, seed=2, iters=14, source=int(gg.pick_sources(g, 1, 2)[0]))
    a = oracle.run(g, app, "gg", alpha0=3, theta0=0.1, **kw)
    b = oracle.run(g, app, "gg", **kw)
    assert np.array_equal(a.values, b.values) and np.array_equal(a.mask, b.mask) and a.edges == b.edges


def test_decoupled_schedule():
    """Supersteps at alpha0 + 1 and then every alpha + 1 iterations."""
    g = gg.rmat(7, 8, seed=23)
    for a0, a in ((0, 3), (5, 1), (2, 2), (6, 0)):
        r = oracle.run(g, "pr", "gg", sigma=0.5, alpha=a, theta=0.1, alpha0=a0, theta0=0.3, iters=20)
        got = [s.iter for s in r.steps if s.superstep]
        want = [i for i in range(1, 21) if i == a0 + 1 or (i > a0 + 1 and (i - a0 - 1) % (a + 1) == 0)]
        assert got == want, (a0, a)


def test_golden_pr_vstatus():
    fx = _load("pr_vstatus_3v.json")
    g, p = _golden_graph(fx), fx["params"]
    r = oracle.Run(g, "pr", "sp", sigma=p["sigma"], iters=p["iters"], vstatus=oracle.VSTATUS_ABS, eps=p["eps"])
    for it in range(1, p["iters"] + 1):
        st = r.step()
        assert np.max(np.abs(r.values() - _fr(fx["expected"]["values_after"][str(it)]))) <= 1e-15, it
        assert st.edges == fx["expected"]["edges_gathered"][str(it)], it
        if str(it) in fx["expected"]["active_after"]:
            assert list(r.vactive()) == fx["expected"]["active_after"][str(it)], it
    # strict comparison: with eps = 0, vertex 2 (1/3 before and after the
    # first iteration) is inactive
    r = oracle.Run(g, "pr", "sp", sigma=1.0, iters=2, vstatus=oracle.VSTATUS_ABS, eps=0.0)
    r.step()
    assert list(r.vactive()) == [1, 1, 0]


def test_vstatus_extremes():
    """A huge epsilon freezes every value after the first iteration (which
    processes every vertex); with epsilon = 0 in accurate iterations nothing
    is skipped, so an exact run is unchanged."""
    g = gg.rmat(9, 8, seed=25)
    one = oracle.run(g, "pr", "exact", iters=1).values
    r = oracle.run(g, "pr", "sp", sigma=0.7, seed=3, iters=8, vstatus=oracle.VSTATUS_ABS, eps=1e9)
    first = oracle.run(g, "pr", "sp", sigma=0.7, seed=3, iters=1)
    assert np.array_equal(r.values, first.values)
    assert r.edges == first.edges
    assert not np.array_equal(first.values, one)  # the first sampled iteration is not the exact one
    a = oracle.run(g, "pr", "exact", iters=6, vstatus=oracle.VSTATUS_REL, eps=0.5)
    b = oracle.run(g, "pr", "exact", iters=6)
    assert np.array_equal(a.values, b.values)


def test_set_mask_replays_flags():
    """Adopting the run's own flags changes nothing; adopting all-ones makes
    the next SP iteration gather every edge and equal an exact iteration."""
    g = gg.rmat(8, 8, seed=27)
    a = oracle.Run(g, "pr", "sp", sigma=0.3, seed=4, iters=3)
    b = oracle.Run(g, "pr", "sp", sigma=0.3, seed=4, iters=3)
    a.step()
    b.step()
    b.set_mask(b.mask())
    sa, sb = a.step(), b.step()
    assert np.array_equal(a.values(), b.values()) and sa.edges == sb.edges
    b.set_mask(np.ones(g.m))
    x = b.values()
    st = b.step()
    assert st.edges == g.m
    e = oracle.Run(g, "pr", "exact", iters=3)
    e.step()
    e.step()
    # one exact iteration from the same state: compare through a fresh exact step on b's input
    outdeg = g.outdeg().astype(np.float64)
    dang = x[outdeg == 0].sum()
    want = np.full(g.n, 0.15 / g.n) + 0.85 * (np.bincount(g.dst(), weights=x[g.col] / outdeg[g.col],
                                                          minlength=g.n) + dang / g.n)
    assert np.max(np.abs(b.values() - want)) <= 1e-15


# --------------------------------------------------------------------------
# Belief propagation (the reading: binary pairwise MRF, messages from the
# sender's belief, value = belief log-odds)
# --------------------------------------------------------------------------

def _ev(expr):
    """Value of a closed-form expression of the golden files (ln, products, quotients)."""
    return float(eval(expr, {"__builtins__": {}}, {"ln": math.log}))


@pytest.mark.parametrize("case", ["pos", "neg"])
def test_golden_bp_superstep(case):
    """Hand-worked GG run on 3 vertices: values after every iteration, the
    influences and flags of the superstep (closed forms, tests/golden)."""
    fx = json.load(open(os.path.join(GOLDEN, "bp_superstep_3v.json")))
    g, p = _golden_graph(fx), fx["params"]
    c = fx["cases"][case]
    prior = np.array([_ev(x) for x in c["prior"]])
    r = oracle.Run(g, "bp", p["policy"], sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], seed=1,
                   iters=p["iters"], coupling=p["coupling"], prior=prior)
    for it in range(1, p["iters"] + 1):
        info = r.step()
        want = np.array([_ev(x) for x in c["values_after"][str(it)]])
        assert np.allclose(r.values(), want, rtol=1e-12, atol=1e-12), (it, r.values(), want)
        if info.superstep:
            infl = r.influence()
            want_i = np.array([_ev(x) for x in c["influence_at_superstep_2"]])
            assert np.allclose(infl, want_i, rtol=1e-6), (infl, want_i)  # binary32-rounded messages
            assert r.mask().tolist() == c["mask_after_superstep_2"]
    r.close()


@pytest.mark.parametrize("kappa", [0.0, 0.1, 0.6, 0.95])
def test_bp_message_closed_form(kappa):
    """The message from the definition (sum over the sender's states of the
    potential times its belief) equals the closed form 2 atanh(kappa tanh(L/2)),
    is odd in L, zero at L = 0 and bounded by 2 atanh(kappa)."""
    for L in (-40.0, -5.0, -1.0, -0.3, 0.0, 1e-9, 0.7, 3.0, 12.0, 700.0):
        m = oracle.bp_message(L, kappa)
        want = 2.0 * math.atanh(kappa * math.tanh(L / 2.0))
        assert abs(m - want) <= 1e-12 * max(1.0, abs(want)), (L, m, want)
        assert oracle.bp_message(-L, kappa) == -m
        assert abs(m) <= 2.0 * math.atanh(kappa) + 1e-15
    assert oracle.bp_message(0.0, kappa) == 0.0


def _bp_graph_and_prior(scale=9, seed=31):
    g = gg.rmat(scale, 8, seed=seed, symmetrize=True)
    return g, gg.bp_prior(g.n, seed).astype(np.float64)


def test_bp_zero_coupling_keeps_the_prior():
    g, h = _bp_graph_and_prior()
    r = oracle.run(g, "bp", "exact", iters=7, coupling=0.0, prior=h)
    assert np.array_equal(r.values, h)


def test_bp_graph_without_edges_keeps_the_prior():
    n = 50
    g = gg.Graph(n=n, rowptr=np.zeros(n + 1, dtype=np.int32), col=np.zeros(0, dtype=np.int32))
    h = gg.bp_prior(n, 5).astype(np.float64)
    r = oracle.run(g, "bp", "exact", iters=5, coupling=0.7, prior=h)
    assert np.array_equal(r.values, h)


def test_bp_single_edge():
    """v -> u: after any number of iterations u holds its prior plus v's
    message, v (no in-edge) its prior."""
    g = gg.from_edges(2, [0], [1])
    h = np.array([1.3, -0.4])
    for it in (1, 2, 5):
        r = oracle.run(g, "bp", "exact", iters=it, coupling=0.45, prior=h)
        assert r.values[0] == 1.3
        assert abs(r.values[1] - (-0.4 + 2 * math.atanh(0.45 * math.tanh(0.65)))) < 1e-14


def test_bp_cycle_converges_to_the_scalar_fixed_point():
    """On a symmetric cycle (in-degree 2) with one prior h everywhere, every
    vertex converges to the root of L = h + 2 * 2 atanh(kappa tanh(L/2)),
    found by scipy's brentq (a contraction for 2 kappa < 1)."""
    from scipy.optimize import brentq
    n, h0, kappa = 12, 0.3, 0.35
    src = list(range(n)) + [(i + 1) % n for i in range(n)]
    dst = [(i + 1) % n for i in range(n)] + list(range(n))
    g = gg.from_edges(n, src, dst)
    r = oracle.run(g, "bp", "exact", iters=300, coupling=kappa, prior=np.full(n, h0))
    f = lambda L: L - h0 - 4.0 * math.atanh(kappa * math.tanh(L / 2.0))
    want = brentq(f, -50.0, 50.0, xtol=1e-15)
    assert np.allclose(r.values, want, rtol=1e-12, atol=1e-12), (r.values[:3], want)


def test_bp_sign_symmetry_and_monotonicity():
    """Negating every prior negates every value (exactly: the message is an
    odd function); raising one prior lowers no vertex's value."""
    g, h = _bp_graph_and_prior()
    a = oracle.run(g, "bp", "exact", iters=6, coupling=0.5, prior=h).values
    b = oracle.run(g, "bp", "exact", iters=6, coupling=0.5, prior=-h).values
    assert np.array_equal(a, -b)
    h2 = h.copy()
    v = int(np.argmax(np.diff(g.rowptr)))
    h2[v] += 2.0
    c = oracle.run(g, "bp", "exact", iters=6, coupling=0.5, prior=h2).values
    assert np.all(c >= a) and c[v] > a[v]


def test_bp_sigma_one_alpha_zero_is_exact():
    """SP with every edge kept and SMS from iteration 1 equal the exact run."""
    g, h = _bp_graph_and_prior()
    ex = oracle.run(g, "bp", "exact", iters=8, coupling=0.4, prior=h).values
    sp = oracle.run(g, "bp", "sp", sigma=1.0, iters=8, coupling=0.4, prior=h).values
    sms = oracle.run(g, "bp", "sms", sigma=0.3, alpha=0, iters=8, coupling=0.4, prior=h).values
    assert np.array_equal(ex, sp) and np.array_equal(ex, sms)


def test_bp_rejects_unsupported():
    g, h = _bp_graph_and_prior()
    with pytest.raises(ValueError):
        oracle.Run(g, "bp", "exact", coupling=1.0, prior=h)
    with pytest.raises(ValueError):
        oracle.Run(g, "bp", "exact", coupling=0.5)
    with pytest.raises(ValueError):
        oracle.Run(g, "bp", "gg", coupling=0.5, prior=h, influence=oracle.INFL_TOTAL)


# --------------------------------------------------------------------------
# Influence in push order (SSSP/CC): the running value starts at the
# destination's own value
# --------------------------------------------------------------------------

def _inf_list(v):
    return [0xFFFFFFFF if x == "INF" else x for x in v]


def test_golden_sssp_push_influence():
    fx = _load("sssp_push_influence_4v.json")
    e = fx["graph"]["edges"]
    g = gg.from_edges(4, [x[0] for x in e], [x[1] for x in e], [x[2] for x in e])
    p = fx["params"]
    r = oracle.Run(g, "sssp", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], source=p["source"],
                   iters=p["iters"], influence=oracle.INFL_PUSH)
    gathered = []
    for it in range(1, p["iters"] + 1):
        st = r.step()
        gathered.append(st.edges)
        assert r.values().tolist() == _inf_list(fx["expected"]["values_after"][str(it)]), it
        if str(it) in fx["expected"]["mask_after"]:
            assert r.mask().tolist() == fx["expected"]["mask_after"][str(it)], it
    assert gathered == fx["expected"]["edges_gathered"]
    r.close()


def test_golden_cc_push_influence():
    fx = _load("cc_push_influence_path3.json")
    e = fx["graph"]["edges"]
    g = gg.from_edges(3, [x[0] for x in e], [x[1] for x in e])
    p = fx["params"]
    for infl, key in ((oracle.INFL_PUSH, "mask_after_superstep_2"), (oracle.INFL_PREFIX, "prefix_mask_after_superstep_2")):
        r = oracle.Run(g, "cc", "gg", sigma=p["sigma"], alpha=p["alpha"], theta=p["theta"], iters=p["iters"],
                       influence=infl)
        for it in range(1, p["iters"] + 1):
            r.step()
            assert r.values().tolist() == fx["expected"]["values_after"][str(it)], it
            if it == 2:
                assert r.mask().tolist() == fx["expected"][key]
        r.close()


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_push_flags_are_a_subset_of_prefix_flags(app):
    """From the same state (identical runs up to the first superstep), an
    edge active in push order is active under PREFIX too: its running value
    is never above PREFIX's, so it improves it less. The subset is strict on
    R-MAT, and values are unaffected by the flags of that superstep."""
    g = gg.rmat(10, 8, seed=12, weights=(app == "sssp"), symmetrize=(app == "cc"))
    cand = gg.pick_sources(g, 8, 12)
    s = int(cand[np.argmax(g.outdeg()[cand])])
    runs = {}
    for infl in (oracle.INFL_PREFIX, oracle.INFL_PUSH):
        r = oracle.Run(g, app, "gg", sigma=0.5, alpha=7, theta=0.05, seed=2, source=s, iters=8, influence=infl)
        for _ in range(8):
            r.step()
        runs[infl] = (r.mask(), r.values())
        r.close()
    mp, vp = runs[oracle.INFL_PREFIX]
    mu, vu = runs[oracle.INFL_PUSH]
    assert np.all(mu <= mp) and mu.sum() < mp.sum()
    assert np.array_equal(vp, vu)


def test_push_influence_rejected_for_sum_apps():
    g = gg.rmat(6, 4, seed=1)
    for app in ("pr", "ppr"):
        with pytest.raises(ValueError):
            oracle.Run(g, app, "gg", influence=oracle.INFL_PUSH)
