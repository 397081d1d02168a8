"""GPU parity of the learned-correction pieces with the CPU oracle: the MLP's
forward pass, loss gradient and Adam step (same bfloat16 weights and
features, oracle in binary64 with the kernels' rounding points), the
per-vertex features and drift labels of traced supersteps, and whole LEARNED
runs whose selections the two sides make identically.

Tolerances. Logits: binary32 accumulation of at most 64-term dot products
differs from the binary64 sums by a few 1e-7 relative; where that moves a
hidden activation across a bfloat16 rounding boundary the logit moves by
about 2^-8 of that unit's contribution, which is rare. Gradients: the same
plus binary32 sums over the batch. Exact-weight networks (one nonzero weight
per unit, dyadic values) make every sum exact, so their logits and the
selections they make are identical on both sides.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import (bf16_to_f64, compare_values, graph_for, log, mlp_random_features, mlp_random_params,
                     mlp_selector_params, oracle_kw, rel_l1)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


def dev_bf16(bits):
    import torch
    return torch.from_numpy(np.ascontiguousarray(bits, dtype=np.uint16).view(np.int16)).cuda()


def dev_f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# --------------------------------------------------------------------------
# MLP kernels
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mlp_forward_matches_oracle(P, seed):
    n = 5003  # 313 tiles of 16 with a ragged tail
    p = mlp_random_params(seed)
    f = mlp_random_features(seed + 10, n)
    net = P.Mlp()
    net.set_weights(p.astype(np.float32))
    got = net.forward(dev_bf16(f)).cpu().numpy().astype(np.float64)
    want = oracle.mlp_forward(p, f, rounding=True)
    err = np.abs(got - want) / (1.0 + np.abs(want))
    log("forward seed", seed, "median", np.median(err), "p99.9", np.quantile(err, 0.999), "max", err.max())
    assert np.median(err) < 1e-6
    assert np.quantile(err, 0.999) < 1e-5  # binary32 accumulation only
    assert err.max() < 5e-3  # a hidden activation crossing a bfloat16 rounding boundary
    net.close()


def test_mlp_forward_exact_weights(P):
    """Selector networks compute logit = scale * feature exactly."""
    n = 777
    f = mlp_random_features(5, n)
    net = P.Mlp()
    for k, scale in ((0, 1.0), (2, -2.0), (3, 0.5)):
        net.set_weights(mlp_selector_params(k, scale).astype(np.float32))
        got = net.forward(dev_bf16(f)).cpu().numpy().astype(np.float64)
        want = np.maximum(bf16_to_f64(f[:, k]), 0) * scale
        assert np.array_equal(got, want), k
        assert np.array_equal(got, oracle.mlp_forward(mlp_selector_params(k, scale), f, rounding=True))
    net.close()


@pytest.mark.parametrize("seed", [4, 5])
def test_mlp_grad_matches_oracle(P, seed):
    n = 2999
    p = mlp_random_params(seed)
    f = mlp_random_features(seed + 20, n)
    y = (np.random.default_rng(seed).uniform(size=n) < 0.25).astype(np.float32)
    net = P.Mlp()
    net.set_weights(p.astype(np.float32))
    g = net.loss_grad(dev_bf16(f), dev_f32(y), pos_weight=3.0).cpu().numpy().astype(np.float64)
    loss, want = oracle.mlp_loss_grad(p, f, y, pos_weight=3.0, rounding=True)
    _, pure = oracle.mlp_loss_grad(p, f, y, pos_weight=3.0, rounding=False)
    blocks = {"W1": (oracle.P_W1, oracle.P_B1), "b1": (oracle.P_B1, oracle.P_W2), "W2": (oracle.P_W2, oracle.P_B2),
              "b2": (oracle.P_B2, oracle.P_W3), "w3": (oracle.P_W3, oracle.P_B3), "b3": (oracle.P_B3, oracle.MLP_PARAMS)}
    for name, (a, b) in blocks.items():
        d = np.linalg.norm(g[a:b] - want[a:b]) / max(np.linalg.norm(want[a:b]), 1e-30)
        dp = np.linalg.norm(g[a:b] - pure[a:b]) / max(np.linalg.norm(pure[a:b]), 1e-30)
        log("grad", name, "rel L2 vs rounded oracle %.2e, vs binary64 %.2e" % (d, dp))
        assert d < 2e-5, name  # binary32 sums over the batch
        assert dp < 5e-2, name  # the bfloat16 rounding points themselves
    assert abs(g[oracle.MLP_PARAMS] - loss * n) <= 1e-5 * loss * n
    net.close()


def test_mlp_adam_matches_oracle(P):
    import torch
    p = mlp_random_params(6)
    net = P.Mlp()
    net.set_weights(p.astype(np.float32))
    rng = np.random.default_rng(7)
    po, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for t in range(1, 4):
        g = (rng.normal(size=oracle.MLP_PARAMS) * 1e-2).astype(np.float32).astype(np.float64)
        oracle.adam_step(po, m, v, g, 1e-3, t)
        net.adam_step(torch.from_numpy(g.astype(np.float32)).cuda(), 1e-3)
    got = net.get_weights().astype(np.float64)
    assert np.all(np.abs(got - po) <= 1e-6 + 1e-5 * np.abs(po))
    net.close()


def test_mlp_training_reduces_loss(P):
    """Adam on a learnable rule (drift iff delta1 > 0.3 or active fraction < 0.2)."""
    n = 8192
    f = mlp_random_features(8, n)
    x = bf16_to_f64(f)
    y = ((x[:, 3] > 0.3) | (x[:, 2] < 0.2)).astype(np.float32)
    net = P.Mlp(seed=3)
    fd, yd = dev_bf16(f), dev_f32(y)
    first = None
    for it in range(300):
        lo = (it * 1024) % n
        g = net.loss_grad(fd[lo:lo + 1024], yd[lo:lo + 1024], pos_weight=1.0)
        if first is None:
            first = g[oracle.MLP_PARAMS].item() / 1024
        net.adam_step(g, 3e-3)
    last = net.loss_grad(fd, yd)[oracle.MLP_PARAMS].item() / n
    log("training loss %.4f -> %.4f" % (first, last))
    assert last < 0.5 * first
    logits = net.forward(fd).cpu().numpy()
    acc = ((logits > 0) == (y > 0.5)).mean()
    log("training accuracy", acc)
    assert acc > 0.9
    net.close()


# --------------------------------------------------------------------------
# Features, traces and labels of runs
# --------------------------------------------------------------------------

def _pr_delta_close(g, o):
    """PR/PPR delta features: the binary32 values differ from the oracle's by
    about 1e-7 relative, which cancellation in the delta magnifies; allow that
    plus one bfloat16 step."""
    a, b = bf16_to_f64(g), bf16_to_f64(o)
    return np.abs(a - b) <= 2e-5 + 2.0 ** -7 * np.maximum(np.abs(a), np.abs(b))


def _compare_features(app, got, want, ctx):
    if app in ("sssp", "cc"):
        bad = np.nonzero(np.any(got != want, axis=1))[0]
        assert bad.size == 0, "%s: %d rows differ, first %s: %s vs %s" % (
            ctx, bad.size, bad[:3].tolist(), got[bad[:3]].tolist(), want[bad[:3]].tolist())
        return
    assert np.array_equal(got[:, [0, 1, 2, 5, 6, 7]], want[:, [0, 1, 2, 5, 6, 7]]), ctx
    for c in (3, 4):
        ok = _pr_delta_close(got[:, c], want[:, c])
        assert ok.all(), "%s col %d: %d rows" % (ctx, c, (~ok).sum())


def _compare_labels(app, got, want, ctx):
    if app in ("sssp", "cc"):
        assert np.array_equal(got, want), ctx
    else:
        # PR drift labels threshold a binary32 difference: rare flips at the boundary
        assert (got != want).mean() <= 0.005, (ctx, int((got != want).sum()))


@pytest.mark.parametrize("app", ["pr", "ppr", "sssp", "cc"])
def test_trace_features_and_labels_match_oracle(P, app):
    g = graph_for(app, 12, seed=3)
    s = int(gg.pick_sources(g, 1, 4)[0])
    kw = dict(sample_ratio=0.3, alpha=2, theta=0.05, seed=5, source=s, iters=12, stop="fixed_iters")
    G = P.Graph.from_host(g)
    T = P.Trace(10 * g.n)
    R = G.begin(app, kw["sample_ratio"], "gg", trace=T, label_eps=1e-3,
                **{k: v for k, v in kw.items() if k != "sample_ratio"})
    O = oracle.Run(g, app, "gg", sigma=kw["sample_ratio"], trace=True, label_eps=1e-3,
                   **oracle_kw({k: v for k, v in kw.items() if k != "sample_ratio"}))
    feats, labs = [], []
    while True:
        a, b = R.step(), O.step()
        if a is None:
            assert b is None
            break
        assert a["kind"] == P.STEP_KIND[b.kind]
        if a["kind"] == "full":
            _compare_features(app, R.features(), O.features(), "iter %d" % b.iter)
            ol = O.labels()
            _compare_labels(app, R.labels(), ol, "iter %d" % b.iter)
            feats.append(O.features())
            labs.append(ol)
            log(app, "iter", b.iter, "drifted", int(ol.sum()), "of", g.n)
        compare_values(app, R.values(), O.values(), ctx="iter %d" % b.iter)
    info = T.info()
    assert info["size"] == g.n * len(feats) and info["dropped"] == 0
    tf, tl = T.export()
    _compare_features(app, tf, np.concatenate(feats), "trace")
    _compare_labels(app, tl.astype(np.uint8), np.concatenate(labs), "trace")
    assert info["positives"] == int(tl.sum())
    R.close()
    T.close()
    G.close()


def test_trace_capacity_drops(P):
    g = graph_for("sssp", 10, seed=2)
    G = P.Graph.from_host(g)
    T = P.Trace(g.n + 100)
    G.approx_run("sssp", 0.3, "gg", alpha=1, theta=0.05, iters=6, source=0, trace=T)
    info = T.info()
    assert info["size"] == g.n + 100 and info["dropped"] == 2 * g.n - 100
    T.clear()
    assert T.info()["size"] == 0
    T.close()
    G.close()


# --------------------------------------------------------------------------
# LEARNED runs
# --------------------------------------------------------------------------

def learned_step_compare(P, g, app, params, tau, rho=1.0, fallback_k=0, audit=False, tuning=None, **kw):
    """Both sides step by step; selections, step kinds, edges, values and
    (after every correction) the flags must agree."""
    net = P.Mlp()
    net.set_weights(params.astype(np.float32))
    G = P.Graph.from_host(g)
    if tuning:
        G.set_tuning(**tuning)
    sr = kw.pop("sample_ratio")
    R = G.begin(app, sr, "learned", mlp=net, tau=tau, rho=rho, fallback_k=fallback_k, audit=audit, **kw)
    O = oracle.Run(g, app, "learned", sigma=sr, mlp=params, tau=tau, rho=rho, fallback_k=fallback_k,
                   trace=audit, **oracle_kw(kw))
    kinds = []
    hits = pos = 0
    while True:
        a, b = R.step(), O.step()
        if a is None:
            assert b is None
            break
        kinds.append(a["kind"])
        assert a["kind"] == P.STEP_KIND[b.kind], (a, b)
        assert a["selected"] == b.selected, (a, b)
        assert a["edges"] == b.edges, (a, b)
        if a["kind"] == "partial":
            # the selected rows are read once, by the superstep
            assert a["edges_processed"] == a["edges"], a
        if app in ("sssp", "cc"):
            assert a["changed"] == b.changed, (a, b)
        if a["selected"] >= 0:
            gs, _ = R.selection()
            os_, _ = O.selection()
            assert np.array_equal(gs, os_)
        if a["superstep"]:
            assert np.array_equal(R.mask(), O.mask()), "flags after iteration %d" % b.iter
        if audit and a["kind"] == "full" and a["selected"] >= 0:
            ol = O.labels()
            pos += int(ol.sum())
            hits += int((ol & O.selection()[0]).sum())
        compare_values(app, R.values(), O.values(), ctx="iter %d" % b.iter)
    st = R.stats()
    if audit:
        assert st.audit_positives == pos and st.audit_hits == hits
    R.close()
    G.close()
    net.close()
    return kinds, st


@pytest.mark.parametrize("app", ["pr", "ppr", "sssp", "cc"])
def test_learned_selector_indegree(P, app):
    """Selection by in-degree (f1 = lg(1 + in-degree) > 3, in-degree >= 8)."""
    g = graph_for(app, 12, seed=6)
    s = int(gg.pick_sources(g, 1, 7)[0])
    for fk in (0, 3):
        kinds, st = learned_step_compare(P, g, app, mlp_selector_params(1), tau=3.0, fallback_k=fk,
                                         sample_ratio=0.3, alpha=2, theta=0.05, seed=8, source=s, iters=15)
        assert "partial" in kinds
        assert ("full" in kinds) == (fk > 0)
        log(app, "fallback", fk, "kinds", "".join(k[0] for k in kinds), "partials", st.partial_supersteps)


PARTIAL_TUNINGS = [
    # unsegmented gathers: team rows, wavefront rows, multi-chunk hub rows
    dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=0, seg_vertices=0, frontier_enable=1,
         frontier_div=16),
    # segmented gathers with many segments: hub pieces, wave-row batches
    dict(small_max=4, small_team=4, wave_max=32, hub_chunk=256, seg_enable=1, seg_vertices=64, frontier_enable=1,
         frontier_div=1),
]


@pytest.mark.parametrize("ti", range(len(PARTIAL_TUNINGS)))
@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_learned_partial_tunings(P, app, ti):
    """Partial supersteps over every bin of both gather paths: the
    approximate pass skips the selected rows, the superstep computes them."""
    g = graph_for(app, 12, seed=6)
    s = int(gg.pick_sources(g, 1, 7)[0])
    log("case: partial supersteps", app, PARTIAL_TUNINGS[ti])
    kinds, st = learned_step_compare(P, g, app, mlp_selector_params(1), tau=3.0, tuning=PARTIAL_TUNINGS[ti],
                                     sample_ratio=0.3, alpha=2, theta=0.05, seed=8, source=s, iters=15)
    assert "partial" in kinds and st.partial_supersteps > 0


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_learned_selector_dynamic(P, app):
    """Selections that change over the run: by active fraction (f2 < 0.5,
    via a negative scale) and by the last delta (f3 > 0)."""
    g = graph_for(app, 12, seed=9)
    s = int(gg.pick_sources(g, 1, 10)[0])
    for params, tau in ((mlp_selector_params(2, -1.0), -0.5), (mlp_selector_params(3, 1.0), 0.0)):
        for stop in ("fixed_iters", "fixed_point"):
            learned_step_compare(P, g, app, params, tau=tau, fallback_k=4, audit=True, sample_ratio=0.3, alpha=1,
                                 theta=0.05, seed=11, source=s, iters=20, stop=stop, max_iters=200)


def test_learned_rho_and_empty_selection(P):
    g = graph_for("sssp", 12, seed=12)
    s = int(gg.pick_sources(g, 1, 13)[0])
    kinds, _ = learned_step_compare(P, g, "sssp", mlp_selector_params(1), tau=-1.0, rho=0.5, sample_ratio=0.3,
                                    alpha=2, theta=0.05, seed=14, source=s, iters=9)
    assert [k for k in kinds if k != "approx"] == ["full"] * 3  # every edge selected > rho m
    kinds, _ = learned_step_compare(P, g, "sssp", mlp_selector_params(1), tau=1e30, sample_ratio=0.3,
                                    alpha=2, theta=0.05, seed=14, source=s, iters=9)
    assert [k for k in kinds if k != "approx"] == ["partial"] * 3  # nothing selected


def test_learned_rho_edge_share(P):
    """The full-superstep fallback triggers on the in-edge share of the
    selected rows (in-degree >= 32 here), on both sides alike."""
    g = gg.rmat(12, 16, seed=24, weights=True)
    indeg = np.diff(g.rowptr)
    eshare = indeg[indeg >= 32].sum() / g.m
    for rho, want in ((eshare - 0.01, "full"), (eshare + 0.01, "partial")):
        kinds, _ = learned_step_compare(P, g, "sssp", mlp_selector_params(1), tau=5.0, rho=rho, sample_ratio=0.3,
                                        alpha=2, theta=0.05, seed=4, source=0, iters=6)
        assert [k for k in kinds if k != "approx"] == [want] * 2


@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_learned_random_network_int_apps(P, app):
    """A random network: logits differ from the oracle's only by rounding, so
    the selections agree unless a logit lies within that rounding of tau;
    the test checks that no selection differs outside a 0.05 band and, when
    none differs at all, that the runs agree bit for bit."""
    g = graph_for(app, 12, seed=15)
    s = int(gg.pick_sources(g, 1, 16)[0])
    params = mlp_random_params(17)
    net = P.Mlp()
    net.set_weights(params.astype(np.float32))
    G = P.Graph.from_host(g)
    kw = dict(alpha=2, theta=0.05, seed=18, source=s, iters=12)
    # tau: the median logit of the first correction step's features (oracle)
    O0 = oracle.Run(g, app, "learned", sigma=0.3, mlp=params, tau=0.0, **oracle_kw(kw))
    for _ in range(3):
        O0.step()
    tau = float(np.median(O0.selection()[1]))
    O0.close()
    R = G.begin(app, 0.3, "learned", mlp=net, tau=tau, **kw)
    O = oracle.Run(g, app, "learned", sigma=0.3, mlp=params, tau=tau, **oracle_kw(kw))
    diverged = False
    while True:
        a, b = R.step(), O.step()
        if a is None:
            break
        if a["selected"] >= 0:
            gs, gl = R.selection()
            os_, ol = O.selection()
            diff = np.nonzero(gs != os_)[0]
            assert np.all(np.abs(ol[diff] - tau) < 0.05), "selection differs away from tau"
            lerr = np.abs(gl.astype(np.float64) - ol) / (1 + np.abs(ol))
            log(app, "iter", b.iter, "selected", a["selected"], "logit err max %.2e" % lerr.max(),
                "selection diffs", diff.size)
            if diff.size:
                diverged = True
                break
        compare_values(app, R.values(), O.values(), ctx="iter %d" % b.iter)
    if diverged:
        log("selections split at a boundary logit; values not compared further")
    R.close()
    O.close()
    G.close()
    net.close()


def test_learned_special_cases_on_gpu(P):
    """LEARNED with a fallback at every correction step is GG; with nothing
    selected and no fallback it is SP (GPU against GPU, bit for bit)."""
    for app in ("pr", "sssp", "cc"):
        g = graph_for(app, 13, seed=19)
        s = int(gg.pick_sources(g, 1, 20)[0])
        G = P.Graph.from_host(g)
        net = P.Mlp(seed=4)
        kw = dict(alpha=3, theta=0.05, seed=21, source=s, iters=13)
        a, sa = G.approx_run(app, 0.3, "learned", mlp=net, tau=0.0, fallback_k=1, **kw)
        b, sb = G.approx_run(app, 0.3, "gg", **kw)
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()) and sa.edges_gathered == sb.edges_gathered
        a, sa = G.approx_run(app, 0.3, "learned", mlp=net, tau=1e30, **kw)
        b, sb = G.approx_run(app, 0.3, "sp", **kw)
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()) and sa.edges_gathered == sb.edges_gathered
        net.close()
        G.close()


def test_learned_invalid_args(P):
    g = graph_for("pr", 10, seed=1)
    G = P.Graph.from_host(g)
    with pytest.raises(P.GGError):
        G.approx_run("pr", 0.3, "learned")  # no network
    net = P.Mlp()
    with pytest.raises(P.GGError):
        G.approx_run("pr", 0.3, "learned", mlp=net, fallback_k=-1)
    with pytest.raises(P.GGError):
        G.approx_run("pr", 0.3, "learned", mlp=net, rho=-1.0)
    T = P.Trace(10)
    with pytest.raises(P.GGError):
        G.approx_run("pr", 0.3, "sp", trace=T)  # traces come from GG / LEARNED
    with pytest.raises(P.GGError):
        net.train(T)  # empty trace
    net.close()
    T.close()
    G.close()


def test_train_on_traces(P):
    """Traces from GG runs on one graph, gg_mlp_train over them: the loss
    falls and the trained network is finite."""
    g = graph_for("pr", 13, seed=22)
    G = P.Graph.from_host(g)
    T = P.Trace(40 * g.n)
    for sg in (0.1, 0.3, 0.5):
        G.approx_run("pr", sg, "gg", alpha=2, theta=0.05, seed=23, iters=15, trace=T, label_eps=1e-3)
    info = T.info()
    log("trace", info)
    assert info["size"] == 15 * g.n and info["positives"] > 0
    net = P.Mlp(seed=5)
    pw = (info["size"] - info["positives"]) / info["positives"]
    losses = net.train(T, epochs=4, batch=4096, lr=2e-3, pos_weight=pw, seed=6)
    log("epoch losses", losses.tolist())
    assert np.all(np.isfinite(losses)) and losses[-1] < losses[0]
    assert np.all(np.isfinite(net.get_weights()))
    net.close()
    T.close()
    G.close()
