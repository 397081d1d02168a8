"""Multi-graph batch: many independent graphs run as one block-diagonal union
(one launch per iteration for all of them). Each part must equal the CPU
oracle run on that graph alone (its own vertex count, source and sampling
seed + p)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, device_values, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def family(app, count=12):
    return gg.rmat_family(count, scale_range=(5, 11), ef_range=(4, 16), seed0=300, weights=(app == "sssp"),
                          symmetrize=(app == "cc"))


@pytest.mark.parametrize("policy,sigma", [("exact", 1.0), ("gg", 0.5), ("sp", 0.3), ("sms", 0.6)])
@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_parts_match_separate_runs(P, app, policy, sigma):
    gs = family(app)
    U, ps = gg.union(gs)
    srcs = None
    if app == "sssp":
        srcs = np.array([ps[p] + int(gg.pick_sources(gs[p], 1, 40 + p)[0]) for p in range(len(gs))], np.int32)
    G = P.Graph.from_host(U)
    G.set_parts(ps, srcs)
    T = 30
    log("parts case:", app, policy, sigma, "n", U.n, "m", U.m)
    if policy == "exact":
        out, st = G.exact_run(app, iters=20, max_iters=400, source=0)
    else:
        out, st = G.approx_run(app, sigma, policy, alpha=3, theta=0.1, seed=9, iters=(20 if app == "pr" else T),
                               stop="fixed_iters")
    got = device_values(out, app)
    iters = []
    for p, g in enumerate(gs):
        sl = slice(int(ps[p]), int(ps[p + 1]))
        kw = dict(source=0 if srcs is None else int(srcs[p] - ps[p]))
        if app == "pr":
            kw["iters"] = 20
        elif policy != "exact":
            kw["iters"] = T
        if policy != "exact":
            kw.update(sigma=sigma, alpha=3, theta=0.1, seed=9 + p)
        ref = oracle.run(g, app, policy, **kw)
        want = ref.values
        if app == "cc":
            want = want + ps[p]
        compare_values(app, got[sl], want, ctx="part %d" % p)
        iters.append(ref.iterations)
    if policy == "exact" and app != "pr":
        assert st.iterations == max(iters)
    G.close()


def test_parts_reject_crossing_edge(P):
    gs = family("pr", 3)
    U, ps = gg.union(gs)
    col = U.col.copy()
    col[0] = int(ps[-1]) - 1  # an edge from the last part into the first
    G = P.Graph(U.n, U.rowptr, col)
    with pytest.raises(P.GGError) as ei:
        G.set_parts(ps)
    assert ei.value.code == -2
    G.set_parts(None)
    with pytest.raises(P.GGError):
        G.set_parts(np.array([0, 5, U.n + 1], np.int32))


@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_union64_full_size(P, app):
    """The multi-graph workload at full size, as the benchmark runs it (tuning
    from the autotuner): 64 R-MAT graphs of scale 10..18 and edge factor
    8..32 (seeds 100 + g) as one block-diagonal union, exact for 20 PR
    iterations (SSSP and CC until no part changes), every part checked
    against the oracle run on that graph alone."""
    gs = gg.rmat_family(64, scale_range=(10, 18), ef_range=(8, 32), seed0=100, weights=(app == "sssp"),
                        symmetrize=(app == "cc"))
    U, ps = gg.union(gs)
    srcs = None
    if app == "sssp":
        srcs = np.array([ps[k] + int(gg.pick_sources(gs[k], 1, 50 + k)[0]) for k in range(len(gs))], np.int32)
    G = P.Graph.from_host(U)
    G.set_parts(ps, srcs)
    tuning, _ = G.autotune(app, iters=3 if app == "pr" else 20, max_iters=1000, reps=1)
    log("union64", app, "n", U.n, "m", U.m, "tuning", tuning)
    out, st = G.exact_run(app, iters=20, max_iters=1000)
    got = device_values(out, app)
    iters = []
    for p, g in enumerate(gs):
        sl = slice(int(ps[p]), int(ps[p + 1]))
        kw = dict(source=0 if srcs is None else int(srcs[p] - ps[p]), iters=20)
        ref = oracle.run(g, app, "exact", **kw)
        want = ref.values + (ps[p] if app == "cc" else 0)
        compare_values(app, got[sl], want, ctx="part %d (n %d, m %d)" % (p, g.n, g.m))
        iters.append(ref.iterations)
    if app != "pr":
        assert st.iterations == max(iters)
    else:
        # the whole union's static PR schedule as one captured launch, replayed:
        # bit for bit the kernel-by-kernel result
        G.set_capture(True)
        for _ in range(2):
            outc, stc = G.exact_run(app, iters=20, max_iters=1000)
            assert np.array_equal(device_values(outc, app), got) and stc.edges_gathered == st.edges_gathered
        G.set_capture(False)
    G.close()
