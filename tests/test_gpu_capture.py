"""Captured static schedules (gg_graph_set_capture): whole runs of PR, PPR
and BP under EXACT, SP and SMS captured into a HIP graph and replayed must
give bit-identical values and identical statistics to the same runs
launched kernel by kernel, across replays with other work in between, and
after the graph's tuning or edges change."""
import numpy as np
import pytest

import graphgen as gg
from helpers import load, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def _kw(app, g):
    if app == "bp":
        return dict(coupling=0.2, prior=gg.bp_prior(g.n, 3))
    if app == "ppr":
        return dict(source=int(gg.pick_sources(g, 1, 3)[0]))
    return {}


def _run(G, app, policy, kw):
    if policy == "exact":
        out, st = G.exact_run(app, iters=12, **kw)
    else:
        out, st = G.approx_run(app, 0.3, policy, alpha=4, seed=7, iters=12, **kw)
    return out.cpu().numpy().copy(), (st.iterations, st.edges_gathered, st.edges_processed, st.active_edges)


@pytest.mark.parametrize("app", ["pr", "ppr", "bp"])
@pytest.mark.parametrize("policy", ["exact", "sp", "sms"])
def test_captured_runs_equal_eager_runs(P, app, policy):
    g = gg.rmat(14, 16, seed=3, symmetrize=(app == "bp"))
    kw = _kw(app, g)
    G = load(P, g)
    G.set_capture(False)
    ref, ref_st = _run(G, app, policy, kw)
    G.set_capture(True)
    for k in range(4):  # capture, then replays with other work in between
        out, st = _run(G, app, policy, kw)
        assert np.array_equal(out, ref), (app, policy, k)
        assert st == ref_st, (st, ref_st)
        G.exact_run("pr", iters=2)  # an eager run of another schedule
        G.set_capture(False)
        G.approx_run("pr", 0.5, "gg", iters=5)
        G.set_capture(True)
    G.close()


def test_capture_follows_tuning_and_updates(P):
    g = gg.rmat(13, 16, seed=4)
    G = load(P, g)
    tunings = [dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64,
                    frontier_enable=1, frontier_div=1),
               dict(small_max=32, small_team=32, wave_max=64, hub_chunk=512, seg_enable=0, seg_vertices=0,
                    frontier_enable=0, frontier_div=16)]
    for t in tunings:
        G.set_tuning(**t)
        G.set_capture(False)
        ref, _ = _run(G, "pr", "sms", {})
        G.set_capture(True)
        for _ in range(2):
            out, _ = _run(G, "pr", "sms", {})
            assert np.array_equal(out, ref)
    rng = np.random.default_rng(4)
    dst = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.rowptr))
    pick = rng.choice(g.m, size=500, replace=False)
    G.update(g.col[pick], dst[pick], rng.integers(0, g.n, 300), rng.integers(0, g.n, 300))
    G.set_capture(False)
    ref, _ = _run(G, "pr", "exact", {})
    G.set_capture(True)
    for _ in range(2):
        out, _ = _run(G, "pr", "exact", {})
        assert np.array_equal(out, ref)
    G.close()


def test_capture_timing(P):
    """Device time of the exact PageRank run with and without the captured
    schedule (logged; the kernels are the same)."""
    g = gg.rmat(20, 16, seed=5)
    G = load(P, g)
    res = {}
    for cap in (False, True):
        G.set_capture(cap)
        G.exact_run("pr", iters=20)
        res[cap] = sorted(G.exact_run("pr", iters=20)[1].device_ms for _ in range(5))[2]
    log("exact PR R-MAT 20, 20 iterations: %.3f ms kernel by kernel, %.3f ms captured" % (res[False], res[True]))
    assert res[True] > 0
    G.close()
