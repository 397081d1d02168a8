"""Dynamic graphs on the GPU against the CPU oracle.

An update batch (deletions of existing arcs and of pairs that match none,
insertions of random arcs and of copies of deleted ones) is applied to the
library's graph (gg_graph_update / gg_run_update) and to the oracle's
(apply_update / ggo_run_update). The updated CSR must be identical; a run
updated part way (or after it ended) must reset the same vertices, keep the
same flags and continue step by step like the oracle, with the tolerances of
the static tests.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, device_values, graph_for, load, log, step_compare

pytestmark = pytest.mark.gpu

TUNINGS = [
    dict(small_max=32, small_team=4, wave_max=1024, hub_chunk=2048, seg_enable=1, seg_vertices=0,
         frontier_enable=1, frontier_div=16),
    dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64,
         frontier_enable=1, frontier_div=1),
    dict(small_max=32, small_team=32, wave_max=64, hub_chunk=512, seg_enable=0, seg_vertices=0,
         frontier_enable=0, frontier_div=16),
]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def random_batch(g, seed, n_del, n_ins, weighted, symmetric=False):
    rng = np.random.default_rng(seed)
    dst = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.rowptr))
    pick = rng.choice(g.m, size=min(n_del, g.m), replace=False)
    ds, dd = g.col[pick], dst[pick]
    a = rng.integers(0, g.n, n_ins)
    b = rng.integers(0, g.n, n_ins)
    keep = a != b  # no self-loops
    a, b = a[keep], b[keep]
    if symmetric:
        ds, dd = np.concatenate([ds, dd]), np.concatenate([dd, ds])
        a, b = np.concatenate([a, b]), np.concatenate([b, a])
    ds = np.concatenate([ds, [0]])  # a pair that matches nothing (no self-loops exist)
    dd = np.concatenate([dd, [0]])
    is_ = np.concatenate([a, ds[:3]])  # re-insert copies of three deleted arcs
    id_ = np.concatenate([b, dd[:3]])
    iw = rng.integers(1, 256, is_.size) if weighted else None
    return ds, dd, is_, id_, iw


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("device_batch", [False, True])
def test_graph_update_matches_oracle(P, weighted, device_batch):
    import torch
    g = gg.rmat(13, 16, seed=21, weights=weighted)
    batch = random_batch(g, 21, 3000, 2000, weighted)
    want = oracle.apply_update(g, *batch).graph
    G = load(P, g)
    if device_batch:
        batch = tuple(None if a is None else torch.as_tensor(np.asarray(a, dtype=np.int32), device="cuda")
                      for a in batch)
    G.update(*batch)
    rp, col, w = G.csr(weights=weighted)
    assert np.array_equal(rp, want.rowptr) and np.array_equal(col, want.col)
    if weighted:
        assert np.array_equal(w, want.weight)
    assert G.m == want.m
    G.close()


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_runs_on_the_updated_graph(P, app, ti):
    """A graph updated twice, then run from scratch: every derived structure
    (bins, segments, out-CSR, dangling list) follows the new CSR."""
    g = graph_for(app, 13, seed=22)
    G = load(P, g, TUNINGS[ti])
    s = int(gg.pick_sources(g, 1, 22)[0])
    w = app == "sssp"
    if app != "pr":  # build the out-CSR first, so that the update rebuilds it
        G.exact_run(app, source=s)
    cur = g
    for k in range(2):
        b = random_batch(cur, 30 + k, 2000, 1500, w, symmetric=(app == "cc"))
        G.update(*b)
        cur = oracle.apply_update(cur, *b).graph
    log("case: run on updated graph", app, TUNINGS[ti])
    out, st = G.exact_run(app, source=s, iters=12)
    ref = oracle.run(cur, app, "exact", source=s, iters=12)
    compare_values(app, device_values(out, app), ref.values, ctx="exact after updates")
    step_compare(P, cur, app, "gg", graph_obj=G, sample_ratio=0.4, alpha=2, theta=0.05, seed=3, source=s,
                 iters=9)
    G.close()


@pytest.mark.parametrize("app", ["sssp", "cc"])
@pytest.mark.parametrize("ti", range(len(TUNINGS)))
@pytest.mark.parametrize("kind", ["delete", "insert", "both"])
def test_converged_exact_run_repaired(P, app, ti, kind):
    """A converged exact SSSP/CC run, updated: the taint closure (deletions)
    and the frontier seeded from the reset vertices' in-neighbours and the
    inserted arcs' sources continue exactly like the oracle's dense passes."""
    g = graph_for(app, 14, seed=23)
    s = int(gg.pick_sources(g, 1, 23)[0])
    nd, ni = {"delete": (4000, 0), "insert": (0, 3000), "both": (4000, 3000)}[kind]
    b = random_batch(g, 23, nd, ni, app == "sssp", symmetric=(app == "cc"))
    if kind == "insert":
        b = ([], [], b[2], b[3], b[4])
    log("case: repair", app, kind, TUNINGS[ti])
    step_compare(P, g, app, "exact", tuning=TUNINGS[ti], source=s, max_iters=10000,
                 update=dict(at=None, batch=b, more=10000))


@pytest.mark.parametrize("app", ["pr", "ppr", "bp", "sssp", "cc"])
@pytest.mark.parametrize("policy", ["exact", "sms", "gg"])
def test_run_updated_mid_way(P, app, policy):
    g = graph_for(app if app not in ("ppr", "bp") else ("pr" if app == "ppr" else "cc"), 14, seed=24)
    s = int(gg.pick_sources(g, 1, 24)[0])
    kw = dict(source=s, iters=14)
    if app == "bp":
        kw.update(coupling=0.2, prior=gg.bp_prior(g.n, 24))
    if policy != "exact":
        kw.update(sample_ratio=0.3, alpha=3, theta=0.05, seed=5)
    else:
        kw.update(max_iters=40)
    b = random_batch(g, 24, 3000, 3000, app == "sssp", symmetric=(app in ("cc", "bp")))
    log("case: mid-way update", app, policy)
    step_compare(P, g, app, policy, update=dict(at=5, batch=b, more=6), **kw)


def test_update_errors_leave_everything_unchanged(P):
    g = gg.rmat(10, 8, seed=25, weights=True)
    G = load(P, g)
    rp0, col0, w0 = G.csr(weights=True)

    def code(f):
        with pytest.raises(P.GGError) as ei:
            f()
        return ei.value.code

    assert code(lambda: G.update([g.n], [0])) == -2
    assert code(lambda: G.update([], [], [1], [2], [256])) == -2
    assert code(lambda: G.update([], [], [1], [2])) == -1  # weighted graph, no weight
    rp1, col1, w1 = G.csr(weights=True)
    assert np.array_equal(rp0, rp1) and np.array_equal(col0, col1) and np.array_equal(w0, w1)
    R = G.begin("sssp", 0.5, "gg", source=0, iters=6)
    R.step()
    assert code(lambda: G.update([], [], [1], [2], [3])) == -6  # a run is active
    before = R.values()
    assert code(lambda: R.update([-1], [0])) == -2
    assert code(lambda: R.update([], [], [1], [2], [3], more_iters=-1)) == -1
    assert np.array_equal(R.values(), before)
    R.close()
    G.close()
    h = gg.rmat(9, 8, seed=25)
    H = load(P, h)
    R = H.begin("pr", 0.5, "gg", pr_degree="active", iters=4)
    assert code(lambda: R.update([], [], [1], [2])) == -5
    R.close()
    H.close()
    # rows not sorted by source
    rp = np.array([0, 2, 2, 2], dtype=np.int32)
    U = P.Graph(3, rp, np.array([2, 1], dtype=np.int32))
    assert code(lambda: U.update([], [], [0], [1])) == -5
    U.close()


def test_update_to_and_from_an_empty_graph(P):
    g = gg.from_edges(6, [0, 1, 2], [1, 2, 3])
    G = load(P, g)
    G.update([0, 1, 2], [1, 2, 3])
    rp, col, _ = G.csr()
    assert rp.tolist() == [0] * 7 and col.size == 0
    out, _ = G.exact_run("pr", iters=3)
    assert np.allclose(out.cpu().numpy(), 1.0 / 6)
    G.update([], [], [5, 4], [4, 3])
    rp, col, _ = G.csr()
    assert rp.tolist() == [0, 0, 0, 0, 1, 2, 2] and col.tolist() == [4, 5]
    G.close()


def test_update_refusals_for_parts_and_policies(P):
    """Updates of a graph with parts, and of LEARNED, vertex-status and
    ACTIVE-degree runs, are refused (GG_E_UNSUPPORTED) and change nothing."""
    gs = [gg.rmat(6, 4, seed=70 + k) for k in range(3)]
    U, ps = gg.union(gs)
    G = P.Graph.from_host(U)
    G.set_parts(ps)
    with pytest.raises(P.GGError) as ei:
        G.update([], [], [0], [1])
    assert ei.value.code == -5
    G.close()
    g = gg.rmat(9, 8, seed=71)
    G = load(P, g)
    rp0, col0, _ = G.csr()
    net = P.Mlp(seed=1)
    for kw in (dict(policy="learned", mlp=net, tau=0.0), dict(policy="gg", vstatus="rel", eps=1e-3)):
        pol = kw.pop("policy")
        R = G.begin("pr", 0.5, pol, iters=6, **kw)
        R.step()
        with pytest.raises(P.GGError) as ei:
            R.update([], [], [0], [1])
        assert ei.value.code == -5
        R.close()
    rp1, col1, _ = G.csr()
    assert np.array_equal(rp0, rp1) and np.array_equal(col0, col1)
    net.close()
    G.close()


def test_updates_that_grow_and_shrink_the_graph(P):
    """Consecutive updates that add and remove many arcs: the arrays an update
    replaces serve the next update only when large enough. The CSR after each
    update and an exact SSSP run on the result match the oracle."""
    g = gg.rmat(12, 8, seed=26, weights=True)
    G = load(P, g)
    s = int(gg.pick_sources(g, 1, 26)[0])
    G.exact_run("sssp", source=s)  # builds the out-CSR, carried over by every update
    cur = g
    for k, (nd, ni) in enumerate([(100, 20000), (15000, 100), (50, 30000), (30000, 0)]):
        b = random_batch(cur, 40 + k, nd, ni, True)
        G.update(*b)
        cur = oracle.apply_update(cur, *b).graph
        rp, col, w = G.csr(weights=True)
        assert np.array_equal(rp, cur.rowptr) and np.array_equal(col, cur.col) and np.array_equal(w, cur.weight)
        assert G.m == cur.m
        log("case: grow/shrink update", k, "m", cur.m)
        out, _ = G.exact_run("sssp", source=s)
        ref = oracle.run(cur, "sssp", "exact", source=s)
        assert np.array_equal(device_values(out, "sssp"), ref.values)
    G.close()
