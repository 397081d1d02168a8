"""Influence in push order (SSSP/CC) on the GPU against the CPU oracle: the
running minimum of a superstep row starts at the row's own value. Step by
step, bit for bit, over every superstep kernel (team, wavefront, two-pass
and single-pass hub chunks, flat short rows) by the tunings below."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
from helpers import graph_for, load, log, step_compare

pytestmark = pytest.mark.gpu

TUNINGS = [
    dict(small_max=32, small_team=4, wave_max=1024, hub_chunk=2048, seg_enable=1, seg_vertices=0,
         frontier_enable=1, frontier_div=16),
    dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64,
         frontier_enable=1, frontier_div=1),
    dict(small_max=32, small_team=32, wave_max=64, hub_chunk=512, seg_enable=0, seg_vertices=0,
         frontier_enable=0, frontier_div=16),
    dict(small_max=8, small_team=16, wave_max=128, hub_chunk=4096, seg_enable=1, seg_vertices=1000,
         frontier_enable=1, frontier_div=4),
]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_push_influence_steps(P, app, ti):
    g = graph_for(app, 14, seed=41)
    cand = gg.pick_sources(g, 8, 41)
    s = int(cand[np.argmax(g.outdeg()[cand])])
    log("case: push influence", app, TUNINGS[ti])
    for mu in ("replace", "union"):
        step_compare(P, g, app, "gg", tuning=TUNINGS[ti], sample_ratio=0.5, alpha=3, theta=0.05, seed=2, source=s,
                     iters=16, influence="push", mask_update=mu)


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_push_influence_sms_and_fixed_point(P, app):
    g = graph_for(app, 14, seed=42)
    cand = gg.pick_sources(g, 8, 42)
    s = int(cand[np.argmax(g.outdeg()[cand])])
    step_compare(P, g, app, "gg", sample_ratio=0.3, alpha=2, theta=0.1, seed=3, source=s, influence="push",
                 stop="fixed_point", max_iters=200)


def test_push_influence_golden_on_gpu(P):
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    fx = json.load(open(os.path.join(gdir, "sssp_push_influence_4v.json")))
    e = fx["graph"]["edges"]
    g = gg.from_edges(4, [x[0] for x in e], [x[1] for x in e], [x[2] for x in e])
    p = fx["params"]
    G = load(P, g)
    R = G.begin("sssp", p["sigma"], "gg", alpha=p["alpha"], theta=p["theta"], source=p["source"], iters=p["iters"],
                influence="push")
    for it in range(1, p["iters"] + 1):
        R.step()
        want = [0xFFFFFFFF if v == "INF" else v for v in fx["expected"]["values_after"][str(it)]]
        assert R.values().tolist() == want, it
        if str(it) in fx["expected"]["mask_after"]:
            assert R.mask().tolist() == fx["expected"]["mask_after"][str(it)], it
    R.close()
    fx = json.load(open(os.path.join(gdir, "cc_push_influence_path3.json")))
    e = fx["graph"]["edges"]
    g = gg.from_edges(3, [x[0] for x in e], [x[1] for x in e])
    p = fx["params"]
    H = load(P, g)
    R = H.begin("cc", p["sigma"], "gg", alpha=p["alpha"], theta=p["theta"], iters=p["iters"], influence="push")
    for it in range(1, p["iters"] + 1):
        R.step()
        assert R.values().tolist() == fx["expected"]["values_after"][str(it)], it
        if it == 2:
            assert R.mask().tolist() == fx["expected"]["mask_after_superstep_2"]
    R.close()
    G.close()
    H.close()


def test_push_influence_rejected_for_sum_apps(P):
    g = graph_for("pr", 8, seed=43)
    G = load(P, g)
    for app in ("pr", "ppr"):
        with pytest.raises(P.GGError) as ei:
            G.approx_run(app, 0.5, "gg", influence="push")
        assert ei.value.code == -1
    G.close()
