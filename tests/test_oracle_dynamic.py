"""Pins of the oracle's dynamic-graph update (graph after an update batch,
flag maintenance, value maintenance) against things other than itself:
a brute-force construction of the updated graph, scipy's shortest paths and
connected components on the new graph, the PageRank linear solve, and a
hand-worked example in tests/golden."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = 0xFFFFFFFF


def random_batch(g, rng, n_del, n_ins, weighted):
    """Deletions drawn from existing arcs (plus a pair that matches none),
    insertions of random arcs, some duplicating existing ones."""
    dst = g.dst()
    pick = rng.choice(g.m, size=min(n_del, g.m), replace=False)
    del_src = list(g.col[pick]) + [0]
    del_dst = list(dst[pick]) + [0]  # 0 -> 0: no self-loop exists, matches nothing
    ins_src = list(rng.integers(0, g.n, n_ins)) + list(g.col[pick[:3]])
    ins_dst = list(rng.integers(0, g.n, n_ins)) + list(dst[pick[:3]])
    ins_w = list(rng.integers(1, 256, len(ins_src))) if weighted else None
    return del_src, del_dst, ins_src, ins_dst, ins_w


def brute_force_update(g, del_src, del_dst, ins_src, ins_dst, ins_w):
    """Row by row with Python lists: survivors in old order, then insertions
    in batch order, then a stable sort of the row by source."""
    dels = set(zip((int(x) for x in del_src), (int(x) for x in del_dst)))
    rows = []
    for u in range(g.n):
        row = []
        for e in range(g.rowptr[u], g.rowptr[u + 1]):
            if (int(g.col[e]), u) not in dels:
                row.append((int(g.col[e]), None if g.weight is None else int(g.weight[e]), e))
        rows.append(row)
    for j, (s, d) in enumerate(zip(ins_src, ins_dst)):
        rows[int(d)].append((int(s), None if ins_w is None else int(ins_w[j]), -1))
    rowptr, col, w, oon = [0], [], [], []
    for row in rows:
        row = sorted(row, key=lambda t: t[0])
        col += [t[0] for t in row]
        w += [t[1] for t in row]
        oon += [t[2] for t in row]
        rowptr.append(len(col))
    return rowptr, col, w, oon


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("weighted", [False, True])
def test_update_matches_brute_force(seed, weighted):
    g = gg.rmat(8, 4, seed=seed, weights=weighted)
    rng = np.random.default_rng(seed)
    b = random_batch(g, rng, 60, 50, weighted)
    u = oracle.apply_update(g, *b)
    rowptr, col, w, oon = brute_force_update(g, *b)
    assert u.graph.rowptr.tolist() == rowptr
    assert u.graph.col.tolist() == col
    assert u.old_of_new.tolist() == oon
    if weighted:
        assert u.graph.weight.tolist() == w
    # every old arc is either deleted or continued exactly once
    kept = np.sort(u.old_of_new[u.old_of_new >= 0])
    assert kept.tolist() == np.nonzero(u.deleted_old == 0)[0].tolist()


def test_update_rejects_bad_batches():
    g = gg.rmat(6, 4, seed=1, weights=True)
    with pytest.raises(ValueError):
        oracle.apply_update(g, [], [], [1], [2])  # weighted graph, no weight
    with pytest.raises(ValueError):
        oracle.apply_update(g, [], [], [1], [2], [300])
    with pytest.raises(ValueError):
        oracle.apply_update(g, [g.n], [0], [], [], [])
    h = gg.rmat(6, 4, seed=1)
    with pytest.raises(ValueError):
        oracle.apply_update(h, [], [], [1], [2], [3])
    bad = gg.Graph(n=3, rowptr=np.array([0, 0, 0, 2], dtype=np.int32), col=np.array([2, 1], dtype=np.int32))
    with pytest.raises(ValueError):
        oracle.apply_update(bad, [], [], [0], [1])


def _csr_matrix(ug, weighted):
    dst = np.repeat(np.arange(ug.n), np.diff(ug.rowptr))
    data = ug.weight.astype(np.float64) if weighted else np.ones(ug.m)
    # csgraph reads row -> column as source -> destination; keep the lightest parallel arc
    order = np.lexsort((data, dst, ug.col))
    s, d, w = ug.col[order], dst[order], data[order]
    first = np.ones(s.size, dtype=bool)
    first[1:] = (s[1:] != s[:-1]) | (d[1:] != d[:-1])
    return sp.csr_matrix((w[first], (s[first], d[first])), shape=(ug.n, ug.n))


def _dijkstra(ug, source):
    d = csg.dijkstra(_csr_matrix(ug, True), indices=source)
    return np.where(np.isinf(d), INF, d).astype(np.uint64).astype(np.uint32)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_sssp_update_taint_is_sound_and_converges(seed):
    """After deletions, every vertex the closure leaves alone holds its exact
    distance in the graph without the deleted arcs (scipy; the insertions
    can only shorten paths later), the closure is a strict subset, and
    continuing to the fixed point gives scipy's distances on the new graph."""
    g = gg.rmat(10, 8, seed=seed, weights=True)
    s = int(gg.pick_sources(g, 1, seed)[0])
    r = oracle.Run(g, "sssp", "exact", source=s, max_iters=10000)
    while r.step() is not None:
        pass
    rng = np.random.default_rng(seed)
    b = random_batch(g, rng, 400, 100, True)
    upd = oracle.apply_update(g, *b)
    only_del = oracle.apply_update(g, b[0], b[1], [], [], [])
    r.update(upd, more_iters=10000)
    want = _dijkstra(upd.graph, s)
    reset = r.reset_vertices().astype(bool)
    vals = r.values()
    assert 0 < reset.sum() < g.n
    assert np.all(vals[reset] == np.where(np.arange(g.n)[reset] == s, 0, INF))
    assert np.array_equal(vals[~reset], _dijkstra(only_del.graph, s)[~reset])
    while r.step() is not None:
        pass
    assert np.array_equal(r.values(), want)
    r.close()


def test_cc_update_taint_is_sound_and_converges():
    g = gg.rmat(10, 2, seed=5, symmetrize=True)
    r = oracle.Run(g, "cc", "exact", max_iters=10000)
    while r.step() is not None:
        pass
    rng = np.random.default_rng(5)
    dst = g.dst()
    pick = rng.choice(g.m, size=300, replace=False)
    ds, dd = g.col[pick], dst[pick]
    a = rng.integers(0, g.n, 20)
    b = rng.integers(0, g.n, 20)
    dels = (np.concatenate([ds, dd]), np.concatenate([dd, ds]))
    upd = oracle.apply_update(g, *dels, np.concatenate([a, b]), np.concatenate([b, a]))
    r.update(upd, more_iters=10000)

    def min_labels(ug):
        _, lab = csg.connected_components(_csr_matrix(ug, False), directed=True, connection="weak")
        first = np.full(lab.max() + 1, ug.n)
        np.minimum.at(first, lab, np.arange(ug.n))
        return first[lab].astype(np.int32)

    want = min_labels(upd.graph)
    reset = r.reset_vertices().astype(bool)
    assert 0 < reset.sum() < g.n
    assert np.array_equal(r.values()[~reset], min_labels(oracle.apply_update(g, *dels, [], []).graph)[~reset])
    while r.step() is not None:
        pass
    assert np.array_equal(r.values(), want)
    r.close()


def test_golden_sssp_update():
    fx = json.load(open(os.path.join(GOLDEN, "sssp_update_5v.json")))
    a = fx["graph"]["arcs"]
    g = gg.from_edges(fx["graph"]["n"], [x[0] for x in a], [x[1] for x in a], [x[2] for x in a])
    s = fx["graph"]["source"]
    ex = fx["expected"]
    conv = lambda v: [INF if x == "INF" else x for x in v]
    r = oracle.Run(g, "sssp", "exact", source=s, max_iters=100)
    while r.step() is not None:
        pass
    assert r.iterations == ex["iterations_before"]
    assert r.values().tolist() == ex["values_before"]
    d, i = fx["update"]["delete"], fx["update"]["insert"]
    upd = oracle.apply_update(g, [x[0] for x in d], [x[1] for x in d], [x[0] for x in i], [x[1] for x in i],
                              [x[2] for x in i])
    r.update(upd, more_iters=100)
    assert r.reset_vertices().tolist() == ex["reset"]
    assert r.values().tolist() == conv(ex["values_after_update"])
    while r.step() is not None:
        assert r.values().tolist() == ex["values_after"][str(r.iterations)]
    assert r.iterations == ex["iterations_after"]
    r.close()


def test_unconverged_or_approximate_min_runs_restart_after_deletions():
    g = gg.rmat(9, 8, seed=6, weights=True)
    s = int(gg.pick_sources(g, 1, 6)[0])
    upd = oracle.apply_update(g, [g.col[0]], [g.dst()[0]], [], [], [])
    assert upd.deleted_old.sum() >= 1
    for policy, kw in (("exact", dict(max_iters=1000)), ("gg", dict(sigma=0.5, alpha=2, theta=0.1, iters=6))):
        r = oracle.Run(g, "sssp", policy, source=s, **kw)
        r.step()
        r.step()
        r.update(upd, more_iters=3)
        init = np.full(g.n, INF, dtype=np.uint32)
        init[s] = 0
        assert np.array_equal(r.values(), init)
        assert r.reset_vertices().all()
        r.close()
    # insertions alone keep every value
    r = oracle.Run(g, "sssp", "gg", source=s, sigma=0.5, alpha=2, theta=0.1, iters=6)
    r.step()
    before = r.values()
    r.update(oracle.apply_update(g, [], [], [s], [1], [7]), more_iters=2)
    assert np.array_equal(r.values(), before) and not r.reset_vertices().any()
    r.close()


def test_flags_survive_and_inserted_arcs_are_active():
    g = gg.rmat(9, 8, seed=7)
    r = oracle.Run(g, "pr", "gg", sigma=0.3, alpha=2, theta=0.05, iters=9)
    for _ in range(4):
        r.step()
    old_mask = r.mask()
    rng = np.random.default_rng(7)
    upd = oracle.apply_update(g, *random_batch(g, rng, 200, 200, False))
    r.update(upd, more_iters=0)
    new_mask = r.mask()
    cont = upd.old_of_new >= 0
    assert np.array_equal(new_mask[cont], old_mask[upd.old_of_new[cont]])
    assert np.all(new_mask[~cont] == 1)
    assert 0 < old_mask.mean() < 1
    r.close()


def _pr_solve(ug, d=0.85):
    """PageRank fixed point of the updated graph by a dense linear solve
    (uniform dangling mass)."""
    n = ug.n
    od = np.bincount(ug.col, minlength=n).astype(np.float64)
    dst = np.repeat(np.arange(n), np.diff(ug.rowptr))
    A = np.zeros((n, n))
    np.add.at(A, (dst, ug.col), 1.0 / od[ug.col])
    A[:, od == 0] += 1.0 / n
    return np.linalg.solve(np.eye(n) - d * A, np.full(n, (1 - d) / n))


def test_pagerank_continues_to_the_new_fixed_point():
    g = gg.rmat(8, 8, seed=8)
    r = oracle.Run(g, "pr", "exact", iters=30)
    while r.step() is not None:
        pass
    rng = np.random.default_rng(8)
    upd = oracle.apply_update(g, *random_batch(g, rng, 300, 300, False))
    r.update(upd, more_iters=400)
    while r.step() is not None:
        pass
    assert r.iterations == 430
    assert np.max(np.abs(r.values() - _pr_solve(upd.graph))) <= 1e-12


def test_bp_continues_to_the_fresh_fixed_point():
    g = gg.rmat(8, 8, seed=9, symmetrize=True)
    h = gg.bp_prior(g.n, 9)
    rng = np.random.default_rng(9)
    upd = oracle.apply_update(g, *random_batch(g, rng, 300, 300, False))
    r = oracle.Run(g, "bp", "exact", iters=10, coupling=0.05, prior=h)
    while r.step() is not None:
        pass
    r.update(upd, more_iters=200)
    while r.step() is not None:
        pass
    fresh = oracle.run(upd.graph, "bp", "exact", iters=200, coupling=0.05, prior=h).values
    assert np.max(np.abs(r.values() - fresh)) <= 1e-10


def test_update_refusals():
    g = gg.rmat(7, 4, seed=1)
    upd = oracle.apply_update(g, [], [], [0], [1])
    r = oracle.Run(g, "pr", "gg", sigma=0.5, iters=4, pr_degree=oracle.DEGREE_ACTIVE)
    with pytest.raises(ValueError):
        r.update(upd)
    r.close()
    r = oracle.Run(g, "pr", "gg", sigma=0.5, iters=4)
    with pytest.raises(ValueError):
        r.update(upd, more_iters=-1)
    r.close()
