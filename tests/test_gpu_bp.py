"""Belief propagation on the GPU against the CPU oracle.

The model is a binary pairwise Markov random field with one coupling kappa
on every edge and a seeded prior log-odds per vertex (graphgen.bp_prior);
the value of a vertex is its belief log-odds. Beliefs are compared at 1e-6
relative L1 after every iteration (binary32 messages on the GPU, binary64 in
the oracle); edge flags after every superstep are equal except where the
oracle's decision margin lies within the change of that margin between the
two sides' beliefs (tests/helpers.py, bp_flip_justified), in which case the
oracle adopts the GPU's flags. Graphs are symmetrized R-MAT (an undirected
model).
"""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, device_values, load, log, rel_l1, step_compare

pytestmark = pytest.mark.gpu

TUNINGS = [
    dict(small_max=32, small_team=4, wave_max=1024, hub_chunk=2048, seg_enable=1, seg_vertices=0,
         frontier_enable=1, frontier_div=16),
    dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64,
         frontier_enable=1, frontier_div=1),
    dict(small_max=32, small_team=32, wave_max=64, hub_chunk=512, seg_enable=0, seg_vertices=0,
         frontier_enable=0, frontier_div=16),
    dict(small_max=8, small_team=16, wave_max=128, hub_chunk=1024, seg_enable=1, seg_vertices=1000,
         frontier_enable=1, frontier_div=4),
]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def bp_graph(scale, seed, ef=16):
    g = gg.rmat(scale, ef, seed=seed, symmetrize=True)
    return g, gg.bp_prior(g.n, seed)


def test_bp_golden_on_gpu(P):
    """The hand-worked 3-vertex GG run (tests/golden/bp_superstep_3v.json)."""
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    fx = json.load(open(os.path.join(gdir, "bp_superstep_3v.json")))
    ev = lambda x: float(eval(x, {"__builtins__": {}}, {"ln": math.log}))
    e = fx["graph"]["edges"]
    g = gg.from_edges(3, [x[0] for x in e], [x[1] for x in e])
    p = fx["params"]
    G = load(P, g)
    for name, c in fx["cases"].items():
        log("case:", name)
        prior = np.array([ev(x) for x in c["prior"]], dtype=np.float32)
        R = G.begin("bp", p["sigma"], p["policy"], alpha=p["alpha"], theta=p["theta"], iters=p["iters"],
                    coupling=p["coupling"], prior=prior)
        for it in range(1, p["iters"] + 1):
            info = R.step()
            want = np.array([ev(x) for x in c["values_after"][str(it)]])
            assert np.max(np.abs(R.values() - want)) < 1e-6, (name, it, R.values(), want)
            if info["superstep"]:
                assert R.mask().tolist() == c["mask_after_superstep_2"], name
        R.close()
    G.close()


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
@pytest.mark.parametrize("kappa", [0.1, 0.4])
def test_bp_exact_runs(P, ti, kappa):
    g, h = bp_graph(13, 11)
    log("case: exact bp", kappa, TUNINGS[ti])
    G = load(P, g, TUNINGS[ti])
    out, st = G.exact_run("bp", iters=10, coupling=kappa, prior=h)
    ref = oracle.run(g, "bp", "exact", iters=10, coupling=kappa, prior=h)
    err = compare_values("bp", device_values(out, "bp"), ref.values, ctx="exact bp")
    log("rel L1", err)
    assert st.iterations == 10 and st.edges_gathered == ref.edges
    G.close()


@pytest.mark.parametrize("policy", ["sp", "sms", "gg"])
@pytest.mark.parametrize("kappa", [0.1, 0.4])
def test_bp_steps(P, policy, kappa):
    g, h = bp_graph(14, 12)
    log("case: bp steps", policy, kappa)
    st = {}
    worst = step_compare(P, g, "bp", policy, stats=st, sample_ratio=0.3, alpha=3, theta=0.05, seed=2, iters=16,
                         coupling=kappa, prior=h)
    log("worst rel L1 %.3e, flips %d" % (worst, st["flips"]))


@pytest.mark.parametrize("ti", range(1, len(TUNINGS)))
def test_bp_steps_tunings(P, ti):
    g, h = bp_graph(13, 13)
    log("case: bp gg tuning", TUNINGS[ti])
    step_compare(P, g, "bp", "gg", tuning=TUNINGS[ti], sample_ratio=0.5, alpha=2, theta=0.1, seed=3, iters=9,
                 coupling=0.3, prior=h)


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_bp_union_and_thresholds(P, theta):
    g, h = bp_graph(13, 14)
    log("case: bp gg union", theta)
    step_compare(P, g, "bp", "gg", sample_ratio=0.2, alpha=2, theta=theta, seed=4, iters=9, coupling=0.3, prior=h,
                 mask_update="union")
    step_compare(P, g, "bp", "gg", sample_ratio=0.2, alpha=2, theta=theta, seed=4, iters=9, coupling=0.3, prior=h)


def test_bp_whole_run_equals_oracle(P):
    g, h = bp_graph(14, 15)
    G = load(P, g)
    out, st = G.approx_run("bp", 0.3, "gg", alpha=3, theta=0.02, seed=5, iters=12, coupling=0.2, prior=h)
    ref = oracle.run(g, "bp", "gg", sigma=0.3, alpha=3, theta=0.02, seed=5, iters=12, coupling=0.2, prior=h)
    err = rel_l1(device_values(out, "bp"), ref.values)
    log("free-running rel L1 %.3e, edges %d / %d" % (err, st.edges_gathered, ref.edges))
    # free running: a flag flipped within its band changes the edge total by the
    # flag's span; values stay close
    assert err <= 1e-5
    G.close()


def test_bp_graph_without_edges_and_zero_coupling(P):
    n = 1000
    g = gg.Graph(n=n, rowptr=np.zeros(n + 1, dtype=np.int32), col=np.zeros(0, dtype=np.int32))
    h = gg.bp_prior(n, 3)
    G = load(P, g)
    out, _ = G.exact_run("bp", iters=4, coupling=0.5, prior=h)
    assert np.array_equal(out.cpu().numpy(), h)
    G.close()
    g, h = bp_graph(12, 16)
    G = load(P, g)
    out, _ = G.approx_run("bp", 0.5, "gg", alpha=1, theta=0.1, iters=5, coupling=0.0, prior=h)
    assert np.array_equal(out.cpu().numpy(), h)
    G.close()


def test_bp_rejects(P):
    import torch
    g, h = bp_graph(8, 17)
    G = load(P, g)

    def code(f):
        with pytest.raises(P.GGError) as ei:
            f()
        return ei.value.code

    assert code(lambda: G.exact_run("bp", coupling=1.0, prior=h)) == -1
    assert code(lambda: G.exact_run("bp", coupling=-0.1, prior=h)) == -1
    assert code(lambda: G.exact_run("bp", coupling=0.5)) == -1
    assert code(lambda: G.approx_run("bp", 0.5, "gg", coupling=0.5, prior=h, influence="total")) == -1
    assert code(lambda: G.approx_run("bp", 0.5, "gg", coupling=0.5, prior=h, vstatus="abs", eps=0.1)) == -1
    assert code(lambda: G.approx_run("bp", 0.5, "gg", coupling=0.5, prior=h, pr_degree="active")) == -1
    assert code(lambda: G.approx_run("bp", 0.5, "learned", coupling=0.5, prior=h)) == -5
    out = torch.empty(g.n, dtype=torch.float32, device="cuda")
    assert code(lambda: G.exact_run_noalloc("bp", out)) == -5
    assert code(lambda: G.batch_run("bp", [0, 1])) == -5
    R = G.begin("bp", 0.5, "gg", coupling=0.5, prior=h, iters=3)
    R.step()
    assert code(lambda: R.export_state()) == -5
    R.close()
    with pytest.raises(ValueError):
        G.exact_run("bp", coupling=0.5, prior=h[:-1])
    G.close()
