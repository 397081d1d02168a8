"""Checkpoint and resume of step-API runs (gg_run_export_state /
gg_run_import_state), called through the C ABI.

A run stepped to iteration j, exported, ended, and imported into a fresh run
must continue bit for bit as the uninterrupted run: the same values, edge
flags and counters after every later iteration. The uninterrupted runs are
themselves held to the oracle by the parity tests; the last case here also
checks a resumed run's final values against the oracle directly.
"""
import numpy as np
import pytest

import oracle
from helpers import compare_values, graph_for, log, oracle_kw

pytestmark = pytest.mark.gpu

DEFAULT_BINS = dict(small_max=32, small_team=4, wave_max=1024, hub_chunk=2048, seg_enable=1, seg_vertices=0,
                    frontier_enable=1, frontier_div=16)
# many multi-chunk hubs and source segments; push whenever the frontier allows
SMALL_BINS = dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64,
                  frontier_enable=1, frontier_div=1)
E_INVAL, E_UNSUPPORTED, E_STATE = -1, -5, -6


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


@pytest.fixture(scope="module")
def graphs(P):
    out = {}
    for app in ("pr", "sssp", "cc"):
        g = graph_for(app, 14, 11)
        out[app] = (g, P.Graph.from_host(g))
    yield out
    for _, G in out.values():
        G.close()


def run_kw(app, policy, g):
    kw = dict(alpha=3, theta=0.05, seed=5, iters=20, source=int(np.argmax(g.outdeg())))
    if app != "pr":
        kw["stop"] = "fixed_point"
        kw["max_iters"] = 200
    return kw


def trail(R, app):
    """Values, flags and counters after every remaining iteration."""
    out = []
    while True:
        info = R.step()
        if info is None:
            break
        st = R.stats()
        out.append((info["iter"], info["kind"], info["edges"], R.values(), R.mask_bits(), st.supersteps,
                    st.edges_gathered, st.active_edges))
    return out


def assert_same_trail(a, b, ctx):
    assert len(a) == len(b), (ctx, len(a), len(b))
    for x, y in zip(a, b):
        assert x[:3] == y[:3], (ctx, x[:3], y[:3])
        assert np.array_equal(x[3].view(np.uint32), y[3].view(np.uint32)), (ctx, "values", x[0])
        assert np.array_equal(x[4], y[4]), (ctx, "flags", x[0])
        assert x[5:] == y[5:], (ctx, "counters", x[0], x[5:], y[5:])


@pytest.mark.parametrize("tuned", [False, True])
@pytest.mark.parametrize("policy,sigma", [("exact", 1.0), ("gg", 0.3), ("sms", 0.2), ("sp", 0.5)])
@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_resume_continues_bit_for_bit(P, graphs, app, policy, sigma, tuned):
    g, G = graphs[app]
    G.set_tuning(**(SMALL_BINS if tuned else DEFAULT_BINS))
    kw = run_kw(app, policy, g)
    log("case: resume", app, policy, sigma, "small bins" if tuned else "default bins")
    # uninterrupted run: values after each iteration
    R = G.begin(app, sigma, policy, **kw)
    full = trail(R, app)
    R.close()
    assert len(full) >= 4
    for j in (0, 1, len(full) // 2, len(full) - 1, len(full)):
        R = G.begin(app, sigma, policy, **kw)
        for _ in range(j):
            assert R.step() is not None
        state = R.export_state()
        before = (R.values(), R.mask_bits(), R.stats())
        R.close()
        R2 = G.begin(app, sigma, policy, **kw)
        R2.import_state(state)
        # the imported state reads back as it was exported
        assert np.array_equal(R2.values().view(np.uint32), before[0].view(np.uint32)), (app, policy, j)
        assert np.array_equal(R2.mask_bits(), before[1]), (app, policy, j)
        st = R2.stats()
        assert (st.iterations, st.supersteps, st.edges_gathered) == (
            before[2].iterations, before[2].supersteps, before[2].edges_gathered)
        # a re-export of the imported state is the same blob
        assert np.array_equal(R2.export_state(), state)
        rest = trail(R2, app)
        R2.close()
        assert_same_trail(rest, full[j:], "%s %s j=%d" % (app, policy, j))
    G.set_tuning(**DEFAULT_BINS)


def test_resumed_run_matches_oracle(P, graphs):
    g, G = graphs["sssp"]
    kw = run_kw("sssp", "gg", g)
    R = G.begin("sssp", 0.3, "gg", **kw)
    for _ in range(5):
        R.step()
    state = R.export_state()
    R.close()
    R2 = G.begin("sssp", 0.3, "gg", **kw)
    R2.import_state(state)
    while R2.step() is not None:
        pass
    got = R2.values()
    R2.close()
    ref = oracle.run(g, "sssp", "gg", **oracle_kw(dict(kw, sample_ratio=0.3)))
    compare_values("sssp", got, ref.values, ctx="resumed sssp gg")


def test_state_errors(P, graphs):
    g, G = graphs["pr"]
    kw = run_kw("pr", "gg", g)
    R = G.begin("pr", 0.3, "gg", **kw)
    R.step()
    state = R.export_state()
    # a run that has stepped cannot take a state
    with pytest.raises(P.GGError) as e:
        R.import_state(state)
    assert e.value.code == E_STATE
    R.close()
    # another configuration: theta, app parameters, policy
    for other in (dict(kw, theta=0.1), dict(kw, iters=19)):
        R = G.begin("pr", 0.3, "gg", **other)
        with pytest.raises(P.GGError) as e:
            R.import_state(state)
        assert e.value.code == E_INVAL
        R.close()
    R = G.begin("pr", 0.3, "sms", **kw)
    with pytest.raises(P.GGError) as e:
        R.import_state(state)
    assert e.value.code == E_INVAL
    R.close()
    # truncated, oversized and corrupted blobs
    R = G.begin("pr", 0.3, "gg", **kw)
    for bad in (state[:-4], np.concatenate([state, np.zeros(4, np.uint8)]), state[:16]):
        with pytest.raises(P.GGError) as e:
            R.import_state(bad)
        assert e.value.code == E_INVAL
    bad = state.copy()
    bad[0] ^= 0xFF
    with pytest.raises(P.GGError) as e:
        R.import_state(bad)
    assert e.value.code == E_INVAL
    # the failed imports left the run untouched: it still runs as a fresh run
    R.import_state(state)
    while R.step() is not None:
        pass
    R.close()


def test_learned_state_unsupported(P, graphs):
    g, G = graphs["sssp"]
    net = P.Mlp(seed=3)
    R = G.begin("sssp", 0.3, "learned", mlp=net, tau=0.0, **run_kw("sssp", "gg", g))
    with pytest.raises(P.GGError) as e:
        R.export_state()
    assert e.value.code == E_UNSUPPORTED
    with pytest.raises(P.GGError) as e:
        R.import_state(np.zeros(256, np.uint8))
    assert e.value.code == E_UNSUPPORTED
    R.close()
    net.close()


@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_resume_on_a_union_of_graphs(P, app):
    """Resume on a block-diagonal union (per-part vertex counts, dangling
    masses, sources and sampling seeds) continues as the uninterrupted run."""
    import graphgen as gg
    gs = gg.rmat_family(8, scale_range=(6, 11), ef_range=(4, 16), seed0=500, weights=(app == "sssp"),
                        symmetrize=(app == "cc"))
    U, ps = gg.union(gs)
    srcs = None
    if app == "sssp":
        srcs = np.array([ps[p] + int(gg.pick_sources(gs[p], 1, 60 + p)[0]) for p in range(len(gs))], np.int32)
    G = P.Graph.from_host(U)
    G.set_parts(ps, srcs)
    kw = dict(alpha=2, theta=0.1, seed=3, iters=12)
    log("case: resume on parts", app)
    R = G.begin(app, 0.4, "gg", **kw)
    full = trail(R, app)
    R.close()
    for j in (1, 5, len(full) - 1):
        R = G.begin(app, 0.4, "gg", **kw)
        for _ in range(j):
            R.step()
        state = R.export_state()
        R.close()
        R2 = G.begin(app, 0.4, "gg", **kw)
        R2.import_state(state)
        rest = trail(R2, app)
        R2.close()
        assert_same_trail(rest, full[j:], "parts %s j=%d" % (app, j))
    G.close()
