"""The autotuner (gg_graph_autotune): it leaves a valid tuning on the graph,
the tuning it reports, and runs after it still match the CPU oracle (SSSP
and CC bit for bit, PageRank within 1e-6 relative L1), for single runs and
for batches."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, device_values, graph_for, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def _valid(t):
    return (t["small_team"] in (4, 8, 16, 32) and 0 <= t["small_max"] <= t["wave_max"]
            and t["hub_chunk"] >= 256 and t["hub_chunk"] % 256 == 0)


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_autotune_exact_int_apps(P, app):
    g = graph_for(app, 14, seed=21)
    s = int(gg.pick_sources(g, 1, 21)[0])
    G = P.Graph.from_host(g)
    t, ms = G.autotune(app, source=s, reps=1)
    log(app, "autotuned", t, "%.3f ms" % ms)
    assert _valid(t) and ms > 0 and G.get_tuning() == t
    out, _ = G.exact_run(app, source=s)
    ref = oracle.run(g, app, "exact", source=s)
    compare_values(app, device_values(out, app), ref.values, ctx="after autotune")
    out, _ = G.approx_run(app, 0.3, "gg", alpha=2, theta=0.05, seed=3, source=s, iters=ref.iterations)
    ref2 = oracle.run(g, app, "gg", sigma=0.3, alpha=2, theta=0.05, seed=3, source=s, iters=ref.iterations)
    compare_values(app, device_values(out, app), ref2.values, ctx="gg after autotune")
    G.close()


def test_autotune_pr_gg(P):
    """Tuned on a short GG PageRank run (one superstep), checked on a full one."""
    g = gg.rmat(14, 16, seed=22)
    G = P.Graph.from_host(g)
    t, ms = G.autotune("pr", 0.3, "gg", alpha=4, theta=0.05, seed=1, iters=5, reps=1)
    log("pr gg autotuned", t, "%.3f ms" % ms)
    assert _valid(t) and G.get_tuning() == t
    out, st = G.approx_run("pr", 0.3, "gg", alpha=4, theta=0.05, seed=1, iters=20)
    ref = oracle.run(g, "pr", "gg", sigma=0.3, alpha=4, theta=0.05, seed=1, iters=20)
    compare_values("pr", device_values(out, "pr"), ref.values, ctx="pr gg after autotune")
    G.close()


@pytest.mark.parametrize("app", ["ppr", "sssp"])
def test_autotune_batch(P, app):
    """Tuned on a 4-iteration batch of 64 queries; a full batch afterwards
    matches the oracle on sampled queries."""
    g = gg.rmat(12, 16, seed=23, weights=(app == "sssp"))
    srcs = gg.pick_sources(g, 64, 23)
    G = P.Graph.from_host(g)
    pol = dict(stop="fixed_iters") if app == "sssp" else {}
    t, ms = G.autotune(app, sources=srcs, iters=4, reps=1, **pol)
    log(app, "batch autotuned", t, "%.3f ms" % ms)
    assert _valid(t) and G.get_tuning() == t
    out, _ = G.batch_run(app, srcs, iters=20)
    got = out.cpu().numpy()
    if app == "sssp":
        got = got.view(np.uint32)
    for q in (0, 17, 63):
        ref = oracle.run(g, app, "exact", source=int(srcs[q]), iters=20)
        compare_values(app, got[:, q], ref.values, ctx="query %d" % q)
    G.close()


def test_autotune_rejects_bad_input(P):
    g = gg.rmat(10, 8, seed=24, weights=True)
    G = P.Graph.from_host(g)
    before = G.get_tuning()
    with pytest.raises(Exception) as ei:
        G.autotune("sssp", source=0, reps=0)
    assert ei.value.code == -1
    with pytest.raises(Exception) as ei:
        G.autotune("sssp", sources=np.array([0, g.n], dtype=np.int32), iters=2, reps=1)
    assert ei.value.code == -1
    assert G.get_tuning() == before
    G.close()
