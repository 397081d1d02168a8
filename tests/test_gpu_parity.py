"""Parity of the HIP library (called through the C ABI) with the CPU oracle.

SSSP and CC must match bit for bit; PageRank within 1e-6 relative L1 (FP32
values on the GPU against the FP64 oracle). Edge-flag decisions after every
superstep must match exactly. Inputs are seeded synthetic graphs: the
2^14-vertex R-MAT of the small PageRank workload, structured tiny graphs,
and tunings that force every bin (team, wavefront, multi-chunk workgroup)
to be used at small sizes.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, device_values, graph_for, load, log, oracle_kw, rel_l1, step_compare

pytestmark = pytest.mark.gpu

TUNINGS = [
    # default
    dict(small_max=32, small_team=4, wave_max=1024, hub_chunk=2048, seg_enable=1, seg_vertices=0,
         frontier_enable=1, frontier_div=16),
    # the earlier default
    dict(small_max=32, small_team=4, wave_max=512, hub_chunk=2048, seg_enable=1, seg_vertices=0,
         frontier_enable=1, frontier_div=16),
    # many multi-chunk hubs, many source segments (several per die), push whenever the frontier allows
    dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64,
         frontier_enable=1, frontier_div=1),
    dict(small_max=32, small_team=32, wave_max=64, hub_chunk=512, seg_enable=0, seg_vertices=0,
         frontier_enable=0, frontier_div=16),
    dict(small_max=8, small_team=16, wave_max=128, hub_chunk=1024, seg_enable=1, seg_vertices=1000,
         frontier_enable=1, frontier_div=4),
    dict(small_max=16, small_team=8, wave_max=2048, hub_chunk=8192, seg_enable=0, seg_vertices=0,
         frontier_enable=0, frontier_div=16),
]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def lib_run(G, app, policy, **kw):
    if policy == "exact":
        kw = {k: v for k, v in kw.items() if k in ("damping", "iters", "max_iters", "source", "dangling")}
        out, st = G.exact_run(app, **kw)
    else:
        sr = kw.pop("sample_ratio")
        out, st = G.approx_run(app, sr, policy, **kw)
    return device_values(out, app), st


def check_run(P, g, app, policy, tuning=None, ctx="", **kw):
    log("case:", ctx, app, policy, kw, tuning)
    G = load(P, g, tuning)
    got, st = lib_run(G, app, policy, **dict(kw))
    okw = oracle_kw(kw)
    if policy == "exact":
        okw.pop("sigma", None)
    ref = oracle.run(g, app, policy, **okw)
    compare_values(app, got, ref.values, ctx="%s %s %s" % (ctx, app, policy))
    assert st.iterations == ref.iterations, (st.iterations, ref.iterations)
    assert st.edges_gathered == ref.edges, (st.edges_gathered, ref.edges)
    G.close()
    return ref


# ---------------------------------------------------------------------------
# Exact (accurate-mode) runs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("gi", range(len(gg.tiny_family())))
def test_exact_tiny_family(P, gi):
    g = gg.tiny_family()[gi]
    check_run(P, g, "pr", "exact", ctx=g.name)
    s = int(gg.pick_sources(g, 1, gi)[0]) if g.m else 0
    check_run(P, g, "sssp", "exact", ctx=g.name, source=s)
    check_run(P, g, "ppr", "exact", ctx=g.name, source=s)
    gs = gg.from_edges(g.n, g.col, g.dst(), symmetrize=True, name=g.name + "_sym")
    check_run(P, gs, "cc", "exact", ctx=gs.name)


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
@pytest.mark.parametrize("app", ["pr", "sssp", "cc", "ppr"])
def test_exact_rmat14(P, app, ti):
    g = graph_for(app, 14, seed=1)
    s = int(gg.pick_sources(g, 1, 1)[0])
    check_run(P, g, app, "exact", tuning=TUNINGS[ti], ctx="rmat14", source=s)


@pytest.mark.parametrize("seg_vertices", [1500, 700, 520, 400])
def test_segment_geometries(P, seg_vertices):
    """Source-segment counts S of 16, 24, 32 and 48 on R-MAT 14: exact runs
    and GG steps, whose active rows get fresh segment offsets after every
    superstep."""
    tuning = dict(TUNINGS[0], seg_vertices=seg_vertices)
    for app in ("pr", "sssp", "cc"):
        g = graph_for(app, 14, seed=1)
        s = int(gg.pick_sources(g, 1, 1)[0])
        log("case: segments", seg_vertices, app)
        check_run(P, g, app, "exact", tuning=tuning, ctx="rmat14 seg %d" % seg_vertices, source=s)
        step_compare(P, g, app, "gg", tuning=tuning, sample_ratio=0.5, alpha=2, theta=0.05, seed=2, source=s,
                     iters=9)


# ---------------------------------------------------------------------------
# Approximate runs: whole-run outputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("policy", ["sp", "sms", "gg"])
@pytest.mark.parametrize("sigma", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_approx_int_apps_rmat14(P, app, sigma, policy):
    g = graph_for(app, 14, seed=1)
    s = int(gg.pick_sources(g, 1, 1)[0])
    L = oracle.run(g, app, "exact", source=s).iterations
    for stop in ("fixed_iters", "fixed_point"):
        check_run(P, g, app, policy, ctx="rmat14", sample_ratio=sigma, alpha=4, theta=0.05, seed=3, source=s,
                  iters=L, stop=stop, max_iters=400)


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_approx_int_apps_tunings(P, ti):
    for app in ("sssp", "cc"):
        g = graph_for(app, 13, seed=5)
        s = int(gg.pick_sources(g, 1, 5)[0])
        check_run(P, g, app, "gg", tuning=TUNINGS[ti], ctx="rmat13", sample_ratio=0.3, alpha=2, theta=0.1,
                  seed=9, source=s, iters=30, stop="fixed_iters")
        check_run(P, g, app, "gg", tuning=TUNINGS[ti], ctx="rmat13-union", sample_ratio=0.3, alpha=2, theta=0.1,
                  seed=9, source=s, iters=30, stop="fixed_iters", mask_update="union")


# ---------------------------------------------------------------------------
# Step-by-step parity with per-superstep flag comparison
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("theta", [0.05, 0.2])
@pytest.mark.parametrize("policy", ["gg", "sp", "sms"])
def test_pr_steps_rmat14(P, policy, theta):
    g = gg.rmat(14, 16, seed=1)
    worst = step_compare(P, g, "pr", policy, sample_ratio=0.5, alpha=4, theta=theta, seed=1, iters=20)
    log("PR %s theta %.2f worst rel L1 %.3e" % (policy, theta, worst))


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_pr_steps_tunings(P, ti):
    g = gg.rmat(12, 16, seed=2)
    step_compare(P, g, "pr", "gg", tuning=TUNINGS[ti], sample_ratio=0.5, alpha=2, theta=0.1, seed=4, iters=9)
    s = int(gg.pick_sources(g, 1, 2)[0])
    step_compare(P, g, "ppr", "gg", tuning=TUNINGS[ti], sample_ratio=0.5, alpha=2, theta=0.1, seed=4, iters=9,
                 source=s)


@pytest.mark.parametrize("app", ["sssp", "cc"])
@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_int_steps_rmat14(P, app, ti):
    g = graph_for(app, 14, seed=1)
    s = int(gg.pick_sources(g, 1, 1)[0])
    step_compare(P, g, app, "gg", tuning=TUNINGS[ti], sample_ratio=0.5, alpha=4, theta=0.05, seed=2, source=s,
                 iters=25)


@pytest.mark.parametrize("ti", [0, 2, 3])
@pytest.mark.parametrize("app", ["pr", "ppr", "sssp", "cc"])
def test_decoupled_first_superstep_steps(P, app, ti):
    """Decoupled parameters [Sec. 3.4, last paragraph]: the first superstep
    after alpha0 approximate iterations with theta0, later ones every alpha+1
    iterations with theta; compared with the oracle after every iteration."""
    g = graph_for(app if app != "ppr" else "pr", 14, seed=5)
    s = int(gg.pick_sources(g, 1, 5)[0])
    if app in ("pr", "ppr"):
        kw = dict(alpha=3, theta=0.2, alpha0=1, theta0=0.01, iters=20)
    else:
        kw = dict(alpha=4, theta=0.05, alpha0=2, theta0=0.5, iters=25)
    step_compare(P, g, app, "gg", tuning=TUNINGS[ti], sample_ratio=0.3, seed=3, source=s, **kw)


@pytest.mark.parametrize("ti", [0, 2, 3])
@pytest.mark.parametrize("app", ["pr", "ppr"])
def test_total_influence_steps(P, app, ti):
    """TOTAL influence (each edge's contribution over its row's sum) step by
    step against the oracle, flags with the replay check."""
    g = graph_for("pr", 14, seed=6)
    s = int(gg.pick_sources(g, 1, 6)[0])
    st = {}
    step_compare(P, g, app, "gg", tuning=TUNINGS[ti], stats=st, sample_ratio=0.3, alpha=3, theta=0.02, seed=2,
                 source=s, iters=20, influence="total")
    log("TOTAL %s tuning %d: %d flags adopted" % (app, ti, st["flips"]))


def test_total_influence_unsupported_with_learned(P):
    g = graph_for("pr", 8, seed=6)
    G = P.Graph.from_host(g)
    net = P.Mlp()
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 0.5, "learned", influence="total", mlp=net, tau=0.0)
    assert ei.value.code == -5
    net.close()
    G.close()


@pytest.mark.parametrize("policy,vs,eps", [("gg", "abs", 1e-7), ("gg", "rel", 0.01), ("sp", "rel", 0.03),
                                            ("sms", "abs", 2e-8)])
@pytest.mark.parametrize("app", ["pr", "ppr"])
def test_vstatus_steps(P, app, policy, vs, eps):
    """GG-VStatus [Alg. 2]: approximate iterations after the first recompute
    only rows reached by an active in-edge from an active vertex; step by
    step against the oracle, vertex statuses and edge flags with the replay
    check (R-MAT 14, n = 16384: 1/n = 6.1e-5)."""
    g = graph_for("pr", 14, seed=7)
    s = int(gg.pick_sources(g, 1, 7)[0])
    st = {}
    step_compare(P, g, app, policy, stats=st, sample_ratio=0.4, alpha=3, theta=0.05, seed=4, source=s, iters=20,
                 vstatus=vs, eps=eps)
    # the rows skipped by the vertex status show in the edges gathered
    G = P.Graph.from_host(g)
    kw = dict(alpha=3, theta=0.05, seed=4, source=s, iters=20)
    _, with_vs = G.approx_run(app, 0.4, policy, vstatus=vs, eps=eps, **kw)
    _, without = G.approx_run(app, 0.4, policy, **kw)
    G.close()
    log("VStatus %s %s %s eps %g: %d statuses, %d flags adopted; edges %d of %d" % (
        app, policy, vs, eps, st["vflips"], st["flips"], with_vs.edges_gathered, without.edges_gathered))
    assert with_vs.edges_gathered < without.edges_gathered


def test_vstatus_rejects(P):
    g = graph_for("sssp", 8, seed=7)
    G = P.Graph.from_host(g)
    with pytest.raises(P.GGError) as ei:
        G.approx_run("sssp", 0.5, "gg", source=1, vstatus="abs", eps=1.0)
    assert ei.value.code == -1
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 0.5, "gg", vstatus="rel", eps=-1.0)
    assert ei.value.code == -1
    net = P.Mlp()
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 0.5, "learned", mlp=net, vstatus="abs", eps=1e-6)
    assert ei.value.code == -5
    net.close()
    R = G.begin("pr", 0.5, "gg")
    with pytest.raises(P.GGError) as ei:
        R.vstatus()
    assert ei.value.code == -6
    R.close()
    G.close()


@pytest.mark.parametrize("ti", [0, 3])
@pytest.mark.parametrize("policy,dangling", [("gg", "uniform"), ("sp", "uniform"), ("sms", "none")])
@pytest.mark.parametrize("app", ["pr", "ppr"])
def test_active_degree_steps(P, app, policy, dangling, ti):
    """ACTIVE out-degree (PageRank of the sparsified graph in approximate
    iterations, vertices without an active out-edge dangling) step by step
    against the oracle."""
    g = graph_for("pr", 14, seed=8)
    s = int(gg.pick_sources(g, 1, 8)[0])
    step_compare(P, g, app, policy, tuning=TUNINGS[ti], sample_ratio=0.3, alpha=3, theta=0.05, seed=5, source=s,
                 iters=16, pr_degree="active", dangling=dangling)


def test_active_degree_rejects(P):
    g = graph_for("sssp", 8, seed=8)
    G = P.Graph.from_host(g)
    with pytest.raises(P.GGError) as ei:
        G.approx_run("sssp", 0.5, "gg", source=1, pr_degree="active")
    assert ei.value.code == -1
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 0.5, "gg", pr_degree="active", vstatus="abs", eps=1e-6)
    assert ei.value.code == -5
    G.close()


def test_decoupled_rejects_bad_parameters(P):
    g = graph_for("pr", 8, seed=5)
    G = P.Graph.from_host(g)
    for kw in (dict(alpha0=-1), dict(theta0=-0.5), dict(theta0=70000.0)):
        with pytest.raises(P.GGError):
            G.approx_run("pr", 0.5, "gg", **kw)
    with pytest.raises(P.GGError):
        G.approx_run("pr", 0.5, "sms", alpha0=2)  # decoupled parameters belong to GG and LEARNED
    G.close()


# ---------------------------------------------------------------------------
# Edge cases
# ---------------------------------------------------------------------------

def test_graph_without_edges(P):
    g = gg.from_edges(5, [], [], [], name="empty5")
    for app in ("pr", "cc", "sssp"):
        check_run(P, g, app, "exact", ctx="empty", source=0)
        check_run(P, g, app, "gg", ctx="empty", sample_ratio=0.5, alpha=1, theta=0.1, source=0, iters=3)


def test_sigma_extremes_and_zero_iters(P):
    g = gg.rmat(10, 8, seed=3, weights=True)
    s = int(gg.pick_sources(g, 1, 3)[0])
    for sr in (0.0, 1.0):
        check_run(P, g, "pr", "gg", ctx="sigma", sample_ratio=sr, alpha=3, theta=0.1, iters=10)
        check_run(P, g, "sssp", "sp", ctx="sigma", sample_ratio=sr, source=s, iters=12)
    G = load(P, g)
    out, st = G.exact_run("pr", iters=0)
    assert st.iterations == 0
    assert np.allclose(out.cpu().numpy(), 1.0 / g.n)


@pytest.mark.parametrize("app", ["pr", "ppr"])
@pytest.mark.parametrize("policy", ["exact", "gg"])
def test_dangling_none(P, app, policy):
    """The literal GG-Apply (mass of vertices without out-edges dropped, not
    spread): exact runs and GG step by step against the oracle on R-MAT 14,
    where about half the vertices have no out-edge, and exact runs on the
    tiny family."""
    g = graph_for(app, 14, seed=3)
    s = int(gg.pick_sources(g, 1, 3)[0])
    if policy == "exact":
        check_run(P, g, app, "exact", ctx="rmat14 dangling none", source=s, dangling="none", iters=20)
        for tg in gg.tiny_family():
            ts = int(gg.pick_sources(tg, 1, 3)[0]) if tg.m else 0
            check_run(P, tg, app, "exact", ctx=tg.name + " dangling none", source=ts, dangling="none", iters=20)
    else:
        step_compare(P, g, app, "gg", sample_ratio=0.5, alpha=4, theta=0.05, seed=2, iters=20, source=s,
                     dangling="none")


def test_golden_examples_on_gpu(P):
    """The hand-worked examples of tests/golden, run through the library."""
    import json
    import os
    from fractions import Fraction
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    fx = json.load(open(os.path.join(gdir, "sssp_superstep_4v.json")))
    e = fx["graph"]["edges"]
    g = gg.from_edges(4, [x[0] for x in e], [x[1] for x in e], [x[2] for x in e])
    G = load(P, g)
    R = G.begin("sssp", 0.0, "gg", alpha=1, theta=0.5, source=0, iters=6)
    for it in range(1, 7):
        R.step()
        want = [0xFFFFFFFF if v == "INF" else int(v) for v in fx["expected"]["values_after"][str(it)]]
        assert R.values().tolist() == want, it
        if str(it) in fx["expected"]["mask_after"]:
            assert R.mask().tolist() == fx["expected"]["mask_after"][str(it)], it
    R.close()
    fx = json.load(open(os.path.join(gdir, "pr_superstep_4v.json")))
    e = fx["graph"]["edges"]
    g = gg.from_edges(4, [x[0] for x in e], [x[1] for x in e])
    G = load(P, g)
    R = G.begin("pr", 1.0, "gg", alpha=1, theta=0.5, iters=3)
    for it in range(1, 4):
        R.step()
        want = np.array([float(Fraction(v)) for v in fx["expected"]["values_after"][str(it)]])
        assert np.max(np.abs(R.values() - want)) < 1e-7
        if it == 2:
            assert R.mask().tolist() == fx["expected"]["mask_after_superstep_2"]
    R.close()


def test_determinism(P):
    g = gg.rmat(14, 16, seed=1)
    G = load(P, g)
    a, _ = G.approx_run("pr", 0.5, "gg", alpha=4, theta=0.05, seed=1)
    a = a.cpu().numpy().copy()
    b, _ = G.approx_run("pr", 0.5, "gg", alpha=4, theta=0.05, seed=1)
    assert np.array_equal(a, b.cpu().numpy())


def test_abi_errors(P):
    import torch
    g = gg.rmat(8, 4, seed=4)
    # malformed CSR
    bad = g.col.copy()
    bad[3] = g.n + 5
    with pytest.raises(P.GGError) as ei:
        P.Graph(g.n, g.rowptr, bad)
    assert ei.value.code == -2
    rp = g.rowptr.copy()
    rp[5], rp[6] = rp[6], rp[5] - 1
    with pytest.raises(P.GGError) as ei:
        P.Graph(g.n, rp, g.col)
    assert ei.value.code == -2
    G = P.Graph(g.n, g.rowptr, g.col)
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 1.5, "gg")
    assert ei.value.code == -1
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 0.5, "gg", theta=-1)
    assert ei.value.code == -1
    with pytest.raises(P.GGError) as ei:
        G.approx_run("pr", 0.5, "gg", alpha=-2)
    assert ei.value.code == -1
    with pytest.raises(P.GGError) as ei:
        G.exact_run("sssp", source=0)  # no weights
    assert ei.value.code == -1
    with pytest.raises(P.GGError) as ei:
        G.approx_run("cc", 0.5, "gg", influence="total")  # TOTAL is a PageRank influence
    assert ei.value.code == -1
    # outputs untouched on failure
    out = torch.full((g.n,), 7.0, device="cuda")
    with pytest.raises(P.GGError):
        G.approx_run("pr", 2.0, "gg", out=out)
    assert torch.all(out == 7.0)
    # weighted graphs: n <= 2^24 (distances then fit uint32), one more vertex is rejected
    for n_w, code in (((1 << 24) + 1, -2), (1 << 24, 0)):
        rp_w = np.zeros(n_w + 1, dtype=np.int32)
        rp_w[1:] = 1  # row 0 holds one in-edge, from vertex 1
        col_w = np.array([1], dtype=np.int32)
        w_w = np.array([7], dtype=np.int32)
        if code:
            with pytest.raises(P.GGError) as ei:
                P.Graph(n_w, rp_w, col_w, w_w)
            assert ei.value.code == code
        else:
            Gw = P.Graph(n_w, rp_w, col_w, w_w)
            d, _ = Gw.exact_run("sssp", source=1)
            d = d.cpu().numpy().view(np.uint32)
            assert d[1] == 0 and d[0] == 7 and d[2] == 0xFFFFFFFF
            Gw.close()
    # one run at a time per graph
    R = G.begin("pr", 0.5, "gg")
    with pytest.raises(P.GGError) as ei:
        G.begin("pr", 0.5, "gg")
    assert ei.value.code == -6
    R.close()


def _giant_hub_graph(seed):
    """2^16 vertices: vertex 0 has an in-edge from every other vertex (one
    row of 65535 edges, sources ascending), plus 4 random in-edges per other
    vertex."""
    n = 1 << 16
    rng = np.random.default_rng(seed)
    src = np.concatenate([np.arange(1, n), rng.integers(0, n, size=4 * n)]).astype(np.int32)
    dst = np.concatenate([np.zeros(n - 1, dtype=np.int64), rng.integers(1, n, size=4 * n)]).astype(np.int32)
    w = rng.integers(1, 256, size=src.size).astype(np.int32)
    return gg.from_edges(n, src, dst, w, name="giant_hub_%d" % seed)


@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_giant_hub_many_chunks_per_segment(P, app):
    """Single-pass hub chunks on one row of 65535 edges split into 256
    chunks, about four per source segment (1024-vertex segments): the chunks
    of the row must keep their order among equal segments. Supersteps every
    third iteration match the oracle."""
    g = _giant_hub_graph(31)
    if app == "cc":
        g = gg.from_edges(g.n, g.col, g.dst(), symmetrize=True, name=g.name + "_sym")
    tuning = dict(small_max=8, small_team=4, wave_max=128, hub_chunk=256, seg_enable=1, seg_vertices=1024)
    check_run(P, g, app, "gg", tuning=tuning, ctx="giant hub", sample_ratio=0.4, alpha=2, theta=0.02, seed=5,
              source=1, iters=9)


@pytest.mark.parametrize("app", ["pr", "sssp"])
def test_superstep_wait_give_up_is_reported(P, app):
    """Every bounded wait of the single-pass hub chunks forced to give up at
    once (wait limit 0, set from the host; no kernel is made to hang): the
    step that ran the superstep returns GG_E_DEVICE, every kernel exits (the
    next run on the same graph completes), and with the default limit back
    that run matches the oracle bit for bit (SSSP) or within tolerance (PR)."""
    g = _giant_hub_graph(31)
    tuning = dict(small_max=8, small_team=4, wave_max=128, hub_chunk=256, seg_enable=1, seg_vertices=1024)
    kw = dict(alpha=1, theta=0.02, seed=5, source=1, iters=4)
    log("case: forced give-up", app, kw)
    G = load(P, g, tuning)
    G.set_wait_limit(0)
    R = G.begin(app, 0.4, "gg", **kw)
    info = R.step()
    assert info is not None and not info["superstep"]
    with pytest.raises(P.GGError) as ei:
        R.step()
    assert ei.value.code == -4 and "gave up" in str(ei.value)
    R.close()
    G.set_wait_limit(1 << 20)
    got, st = lib_run(G, app, "gg", sample_ratio=0.4, **kw)
    ref = oracle.run(g, app, "gg", sigma=0.4, **kw)
    compare_values(app, got, ref.values, ctx="after give-up")
    assert st.edges_gathered == ref.edges
    G.close()


def test_unsorted_rows_disable_segmentation(P):
    """Rows that list their sources out of ascending order: the graph loads
    with source segmentation off (and it stays off when asked for), and runs
    still match the oracle, which walks every row in CSR order."""
    g0 = gg.rmat(12, 16, seed=9, weights=True)
    rng = np.random.default_rng(9)
    col, w = g0.col.copy(), g0.weight.copy()
    for u in range(g0.n):
        b, e = int(g0.rowptr[u]), int(g0.rowptr[u + 1])
        if e - b > 1:
            perm = b + rng.permutation(e - b)
            col[b:e], w[b:e] = col[perm], w[perm]
    g = gg.Graph(n=g0.n, rowptr=g0.rowptr, col=col, weight=w, name="rmat12_shuffled_rows")
    assert np.any(np.diff(col)[np.diff(np.repeat(np.arange(g.n), np.diff(g.rowptr))) == 0] < 0)
    G = load(P, g)
    assert G.get_tuning()["seg_enable"] == 0
    G.set_tuning(seg_enable=1)
    assert G.get_tuning()["seg_enable"] == 0
    G.close()
    assert load(P, g0).get_tuning()["seg_enable"] == 1
    s = int(gg.pick_sources(g, 1, 9)[0])
    check_run(P, g, "pr", "exact", ctx="shuffled rows")
    check_run(P, g, "pr", "gg", ctx="shuffled rows", sample_ratio=0.4, alpha=2, theta=0.05, seed=3, iters=12)
    check_run(P, g, "sssp", "gg", ctx="shuffled rows", sample_ratio=0.4, alpha=2, theta=0.05, seed=3, source=s,
              iters=12)


def test_retune_same_graph(P):
    """Regression: changing the tuning of a loaded graph (including the number
    of source segments, up and down) re-sizes every scratch array."""
    g = gg.rmat(13, 16, seed=6, weights=True)
    s = int(gg.pick_sources(g, 1, 6)[0])
    G = load(P, g)
    ref_pr = oracle.run(g, "pr", "exact").values
    ref_ss = oracle.run(g, "sssp", "exact", source=s).values
    ref_gg = oracle.run(g, "sssp", "gg", sigma=0.4, alpha=2, theta=0.1, seed=5, source=s, iters=12).values
    seq = [dict(seg_enable=1, seg_vertices=0, small_max=4),
           dict(seg_enable=1, seg_vertices=1024, small_max=4),
           dict(seg_enable=1, seg_vertices=128, small_max=4, wave_max=64, hub_chunk=256),
           dict(seg_enable=0, seg_vertices=0, small_max=32),
           dict(seg_enable=1, seg_vertices=64, small_max=2, wave_max=16, hub_chunk=256),
           dict(seg_enable=1, seg_vertices=0, small_max=16, wave_max=2048, hub_chunk=8192)]
    for t in seq:
        log("retune", t)
        G.set_tuning(**t)
        out, _ = G.exact_run("pr")
        compare_values("pr", device_values(out, "pr"), ref_pr, ctx=str(t))
        out, _ = G.exact_run("sssp", source=s)
        compare_values("sssp", device_values(out, "sssp"), ref_ss, ctx=str(t))
        out, _ = G.approx_run("sssp", 0.4, "gg", alpha=2, theta=0.1, seed=5, source=s, iters=12)
        compare_values("sssp", device_values(out, "sssp"), ref_gg, ctx=str(t))
    G.close()


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_idle_iterations_then_superstep(P, app):
    """Approximate iterations after the sampled edges have converged push from
    an empty frontier and launch nothing; the supersteps that follow still
    match the oracle step by step (values, flags, changed counts)."""
    g = graph_for(app, 14, seed=9)
    s = int(gg.pick_sources(g, 1, 9)[0])
    st = {}
    # windows of 14 approximate iterations: longer than the sampled graph
    # needs to converge on this input
    step_compare(P, g, app, "gg", tuning=dict(frontier_enable=1, frontier_div=1), stats=st, sample_ratio=0.3,
                 alpha=14, theta=0.05, seed=4, source=s, iters=45)
    log(app, "idle iterations", st)
    assert st.get("idle", 0) > 0 and st.get("super_after_idle", 0) > 0


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_frontier_push_used_and_exact(P, app):
    """The frontier path runs (some iterations are pushes) and stays bit-exact,
    for the exact baseline and for the sampled schemes."""
    g = graph_for(app, 14, seed=8)
    s = int(gg.pick_sources(g, 1, 8)[0])
    G = load(P, g, dict(frontier_enable=1, frontier_div=4))
    out, st = G.exact_run(app, source=s)
    ref = oracle.run(g, app, "exact", source=s)
    compare_values(app, device_values(out, app), ref.values, ctx="exact frontier")
    assert st.sparse_iterations > 0 and st.edges_processed < st.edges_gathered
    for pol in ("sp", "sms", "gg"):
        out, st = G.approx_run(app, 0.5, pol, alpha=3, theta=0.1, seed=2, source=s, iters=ref.iterations + 5)
        want = oracle.run(g, app, pol, sigma=0.5, alpha=3, theta=0.1, seed=2, source=s, iters=ref.iterations + 5)
        compare_values(app, device_values(out, app), want.values, ctx=pol)
        assert st.edges_gathered == want.edges
    G.close()


@pytest.mark.parametrize("case", ["sssp_tie", "sssp_unreached", "cc_strict"])
def test_estatus_edge_cases_on_gpu(P, case):
    """Hand-built rows where EStatus sits on its boundary (an SSSP improvement
    that ties theta, an unassessable arc, a zero CC influence at theta = 0):
    the library's flags and values equal the oracle's after every step."""
    if case == "sssp_tie":
        g = gg.from_edges(4, [0, 0, 1, 2], [1, 2, 3, 3], [50, 45, 50, 50], name=case)
        app, kw = "sssp", dict(alpha=1, theta=0.05, iters=2, source=0)
    elif case == "sssp_unreached":
        g = gg.from_edges(4, [0, 1, 2], [1, 2, 3], [1, 1, 1], name=case)
        app, kw = "sssp", dict(alpha=1, theta=0.05, iters=2, source=0)
    else:
        g = gg.from_edges(3, [0, 1, 0, 2, 1, 2], [1, 0, 2, 0, 2, 1], None, name=case)
        app, kw = "cc", dict(alpha=0, theta=0.0, iters=1)
    log("case:", case)
    G = P.Graph.from_host(g)
    R = G.begin(app, 1.0, "gg", seed=1, **kw)
    ref = oracle.Run(g, app, "gg", sigma=1.0, seed=1, **kw)
    while True:
        a, b = R.step(), ref.step()
        assert (a is None) == (b is None)
        if a is None:
            break
        assert np.array_equal(R.mask(), ref.mask()), case
        compare_values(app, device_values(R.values(host=False), app), ref.values(), ctx=case)
    R.close()
    ref.close()
    G.close()
