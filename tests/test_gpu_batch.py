"""Multi-query batch runs (many PPR / SSSP queries in one captured HIP graph):
every query equals the single-query CPU oracle run from its source."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def check_batch(P, g, app, nq, policy="exact", sigma=1.0, tuning=None, n_check=6, **kw):
    G = P.Graph.from_host(g)
    if tuning:
        G.set_tuning(**tuning)
    srcs = gg.pick_sources(g, nq, 77 + nq)
    log("batch case:", g.name, app, nq, policy, sigma, tuning)
    out, st = G.batch_run(app, srcs, sample_ratio=sigma, policy=policy, seed=5, **kw)
    got = out.cpu().numpy()
    if app == "sssp":
        got = got.view(np.uint32)
    rng = np.random.default_rng(nq)
    picks = sorted(set([0, nq - 1] + rng.integers(0, nq, size=n_check).tolist()))
    iters = []
    for q in picks:
        okw = dict(source=int(srcs[q]), iters=kw.get("iters", 20))
        if policy != "exact":
            okw.update(sigma=sigma, seed=5)
        if "alpha" in kw:
            okw["alpha"] = kw["alpha"]
        if kw.get("pr_degree") == "active":
            okw["pr_degree"] = oracle.DEGREE_ACTIVE
        if kw.get("dangling") == "none":
            okw["dangling"] = oracle.DANGLING_NONE
        ref = oracle.run(g, app, policy, **okw)
        compare_values(app, got[:, q], ref.values, ctx="query %d" % q)
        iters.append(ref.iterations)
    if app == "sssp" and policy == "exact":
        assert st.iterations >= max(iters)
    G.close()
    return st


@pytest.mark.parametrize("nq", [1, 64, 70, 256])
def test_batch_ppr_exact(P, nq):
    g = gg.rmat(12, 16, seed=11)
    st = check_batch(P, g, "ppr", nq, iters=20)
    assert st.iterations == 20


@pytest.mark.parametrize("nq", [1, 64, 130])
def test_batch_sssp_exact(P, nq):
    g = gg.rmat(12, 16, seed=12, weights=True)
    check_batch(P, g, "sssp", nq)


def test_batch_exact_sssp_stops_at_the_slowest_query(P):
    g = gg.rmat(11, 8, seed=15, weights=True)
    srcs = gg.pick_sources(g, 40, 3)
    G = P.Graph.from_host(g)
    out, st = G.batch_run("sssp", srcs)
    L = max(oracle.run(g, "sssp", "exact", source=int(s)).iterations for s in srcs)
    assert st.iterations == L


@pytest.mark.parametrize("app", ["ppr", "sssp"])
@pytest.mark.parametrize("sigma", [0.3, 0.8])
def test_batch_sp(P, app, sigma):
    g = gg.rmat(12, 16, seed=13, weights=True)
    check_batch(P, g, app, 96, policy="sp", sigma=sigma, iters=15)


@pytest.mark.parametrize("app", ["ppr", "sssp"])
@pytest.mark.parametrize("alpha", [0, 3, 20])
def test_batch_sms(P, app, alpha):
    """SMS: the shared sample for alpha iterations, every edge after (alpha
    = 0 is exact, alpha >= iters is SP); small hub chunks put hub rows in
    both edge sets."""
    g = gg.rmat(13, 16, seed=17, weights=True)
    st = check_batch(P, g, app, 80, policy="sms", sigma=0.3, alpha=alpha, iters=12,
                     tuning=dict(small_max=8, wave_max=64, hub_chunk=512))
    assert st.iterations == 12
    m = int(g.rowptr[-1])
    if alpha == 0:
        assert st.edges_gathered == 80 * 12 * m
    elif alpha >= 12:
        assert st.edges_gathered == 80 * 12 * st.active_edges < 80 * 12 * m
    else:
        assert 80 * (12 - alpha) * m < st.edges_gathered < 80 * 12 * m


@pytest.mark.parametrize("policy,alpha", [("sms", 0), ("sms", 4), ("sms", 20), ("sp", 0)])
def test_batch_ppr_active_degree(P, policy, alpha):
    """Batched PPR with the ACTIVE out-degree: approximate iterations divide
    by the shared sample's out-degree and spread the mass of the vertices
    without a sampled out-edge; every query equals its single oracle run."""
    g = gg.rmat(13, 16, seed=19)
    check_batch(P, g, "ppr", 80, policy=policy, sigma=0.3, alpha=alpha, iters=12, pr_degree="active",
                tuning=dict(small_max=8, wave_max=64, hub_chunk=512))
    check_batch(P, g, "ppr", 80, policy=policy, sigma=0.3, alpha=alpha, iters=12, pr_degree="active",
                dangling="none")


@pytest.mark.parametrize("app", ["ppr", "sssp"])
def test_batch_hub_chunks(P, app):
    """Small hub chunks force the chunked path and its combine."""
    g = gg.rmat(13, 16, seed=14, weights=True)
    check_batch(P, g, app, 64, tuning=dict(small_max=4, wave_max=16, hub_chunk=256), iters=12)


def test_batch_rejects_bad_input(P):
    g = gg.rmat(8, 4, seed=16, weights=True)
    G = P.Graph.from_host(g)
    with pytest.raises(P.GGError):
        G.batch_run("ppr", [g.n + 1])
    with pytest.raises(P.GGError) as ei:
        G.batch_run("cc", [0])
    assert ei.value.code == -5
    with pytest.raises(P.GGError) as ei:
        G.batch_run("ppr", [0], policy="gg")
    assert ei.value.code == -5


C4_SEED = 5  # R-MAT scale 20 of the batched workload; sources from seed 6


def test_c4_rmat20_batches_full_size(P):
    """The batched workload at full size, in the launch configuration the
    benchmark times (tuning picked by the autotuner on a 3-iteration PPR
    batch): R-MAT 20 with 256 PPR and 256 SSSP queries from the same seeded
    sources, exact and SSSP under SMS (sigma 0.05, alpha 10, the exact
    batch's iteration count). A seeded subset of 32 queries of each exact
    batch, and 8 of the SMS batch, equal single-query oracle runs (PPR within
    1e-6 relative L1, SSSP bit for bit)."""
    g = gg.rmat(20, 16, seed=C4_SEED, weights=True)
    srcs = gg.pick_sources(g, 256, C4_SEED + 1)
    G = P.Graph.from_host(g)
    tuning, _ = G.autotune("ppr", sources=srcs, iters=3, reps=1)
    log("C4 tuning", tuning)
    rng = np.random.default_rng(2024)
    picks = sorted(rng.choice(256, size=32, replace=False).tolist())
    out, st = G.batch_run("ppr", srcs, iters=20)
    got = out.cpu().numpy()
    assert st.iterations == 20
    for q in picks:
        log("C4 PPR query", q, "source", int(srcs[q]))
        ref = oracle.run(g, "ppr", "exact", source=int(srcs[q]), iters=20)
        compare_values("ppr", got[:, q], ref.values, ctx="ppr query %d" % q)
    out, st = G.batch_run("sssp", srcs, max_iters=1000)
    got = out.cpu().numpy().view(np.uint32)
    L = st.iterations
    iters = []
    for q in picks:
        log("C4 SSSP query", q, "source", int(srcs[q]))
        ref = oracle.run(g, "sssp", "exact", source=int(srcs[q]))
        compare_values("sssp", got[:, q], ref.values, ctx="sssp query %d" % q)
        iters.append(ref.iterations)
    assert L >= max(iters)
    out, st = G.batch_run("sssp", srcs, sample_ratio=0.05, policy="sms", alpha=10, iters=L, seed=1)
    got = out.cpu().numpy().view(np.uint32)
    for q in picks[:8]:
        log("C4 SSSP SMS query", q)
        ref = oracle.run(g, "sssp", "sms", source=int(srcs[q]), sigma=0.05, alpha=10, iters=L, seed=1)
        compare_values("sssp", got[:, q], ref.values, ctx="sms query %d" % q)
    G.close()
