"""Shared helpers for the GPU parity tests (comparison of the HIP library
with the CPU oracle on identical seeded inputs)."""
import sys

import numpy as np

import graphgen as gg
import oracle

PR_TOL = 1e-6  # relative L1, FP32 GPU against the FP64 oracle
# Replay band: a PageRank edge flag may differ between the two sides only
# when the oracle's influence lies within this relative distance of theta.
# The GPU decides on binary32 contributions of its own binary32 iterate,
# summed in binary64 in another order; the oracle on binary32 roundings of
# its binary64 iterate. Contributions then differ by about one binary32 ulp
# (6e-8 relative), far inside the band.
REPLAY_BAND = 1e-4
# Vertex-status replay band (GG-VStatus): a vertex's status may differ only
# when the oracle's |x_new - x_old| lies within this many times the larger of
# the two values of the bound; the GPU's iterate is binary32 (6e-8 relative).
VSTATUS_BAND = 1e-6


def bp_flip_justified(g, flips, lo_prev, lg_prev, kappa, theta):
    """Replay check of BP edge flags that differ after a superstep.

    Both sides decide |c_e| > theta |P_e| (c_e the binary32 message of the
    edge's source, P_e the running sum of its row up to and including e) on
    their own beliefs of the previous iteration. A flag may differ only where
    the oracle's decision margin |c_e| - theta |P_e| is within four times the
    change of that margin between the two sides' beliefs (the GPU's given as
    its binary32 output), plus a relative 1e-4 theta |P_e| and a rounding
    term 1e-6 (|c_e| + theta S_e), S_e the running sum of |c|. Returns the
    edges that fail the check."""
    bad = []
    rowptr, col = np.asarray(g.rowptr), np.asarray(g.col)
    msg = lambda L: (2.0 * np.arctanh(kappa * np.tanh(0.5 * np.asarray(L, dtype=np.float64)))).astype(np.float32)
    for e in np.asarray(flips).tolist():
        u = int(np.searchsorted(rowptr, e, side="right") - 1)
        src = col[rowptr[u]:e + 1]
        margins = []
        for L in (lo_prev, lg_prev):
            c = msg(L[src]).astype(np.float64)
            P = c.sum()
            margins.append((abs(c[-1]) - theta * abs(P), abs(c[-1]), abs(P), np.abs(c).sum()))
        (mo, co, po, so), (mg, _, _, _) = margins
        allow = 4.0 * abs(mo - mg) + REPLAY_BAND * theta * po + 1e-6 * (co + theta * so)
        if abs(mo) > allow:
            bad.append((e, mo, mg, allow))
    return bad


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l1(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a - b).sum())


def as_u32(x):
    x = np.asarray(x)
    if x.dtype == np.uint32:
        return x
    return x.astype(np.int64).astype(np.uint32) if x.dtype != np.int32 else x.view(np.uint32)


def device_values(t, app):
    """Device tensor from the library -> numpy with the oracle's dtype."""
    h = t.cpu().numpy()
    if app == "sssp":
        return h.view(np.uint32)
    if app == "cc":
        return h.astype(np.int32)
    return h.astype(np.float64)


def compare_values(app, got, want, ctx=""):
    if app in ("pr", "ppr", "bp"):
        err = rel_l1(got, want)
        assert err <= PR_TOL, "%s rel L1 %.3e > %.0e" % (ctx, err, PR_TOL)
        return err
    got = np.asarray(got)
    want = np.asarray(want)
    if app == "sssp":
        got, want = as_u32(got), as_u32(want)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%s: %d mismatches, first %s: got %s want %s" % (
        ctx, bad.size, bad[:5].tolist(), got[bad[:5]].tolist(), want[bad[:5]].tolist())
    return 0.0


def oracle_kw(kw):
    """Translate library keyword arguments to the oracle's."""
    o = dict(kw)
    stop = o.pop("stop", "fixed_iters")
    o["stop"] = oracle.FIXED_POINT if stop == "fixed_point" else oracle.FIXED_ITERS
    mu = o.pop("mask_update", "replace")
    o["mask_update"] = oracle.MASK_UNION if mu == "union" else oracle.MASK_REPLACE
    dg = o.pop("dangling", "uniform")
    o["dangling"] = oracle.DANGLING_NONE if dg == "none" else oracle.DANGLING_UNIFORM
    o["influence"] = {"prefix": oracle.INFL_PREFIX, "total": oracle.INFL_TOTAL,
                      "push": oracle.INFL_PUSH}[o.pop("influence", "prefix")]
    o["pr_degree"] = oracle.DEGREE_ACTIVE if o.pop("pr_degree", "full") == "active" else oracle.DEGREE_FULL
    o["vstatus"] = {"none": oracle.VSTATUS_NONE, "abs": oracle.VSTATUS_ABS,
                    "rel": oracle.VSTATUS_REL}[o.pop("vstatus", "none")]
    if "sample_ratio" in o:
        o["sigma"] = o.pop("sample_ratio")
    return o


def graph_for(app, scale, seed, ef=16):
    if app == "cc":
        return gg.rmat(scale, ef, seed=seed, symmetrize=True)
    return gg.rmat(scale, ef, seed=seed, weights=(app == "sssp"))


# ---------------------------------------------------------------------------
# MLP parameters and features for the learned-policy tests
# ---------------------------------------------------------------------------

def mlp_random_params(seed, scale=1.0):
    """He-uniform weights, small biases; binary32 values in float64."""
    import math
    H, IN = oracle.MLP_HIDDEN, oracle.MLP_IN
    rng = np.random.default_rng(seed)
    p = np.zeros(oracle.MLP_PARAMS)
    p[oracle.P_W1:oracle.P_B1] = rng.uniform(-1, 1, IN * H) * math.sqrt(6.0 / IN) * scale
    p[oracle.P_B1:oracle.P_W2] = rng.uniform(-0.1, 0.1, H)
    p[oracle.P_W2:oracle.P_B2] = rng.uniform(-1, 1, H * H) * math.sqrt(6.0 / H) * scale
    p[oracle.P_B2:oracle.P_W3] = rng.uniform(-0.1, 0.1, H)
    p[oracle.P_W3:oracle.P_B3] = rng.uniform(-1, 1, H) * math.sqrt(6.0 / H) * scale
    p[oracle.P_B3] = 0.05
    return p.astype(np.float32).astype(np.float64)


def mlp_random_features(seed, n):
    """bfloat16 bits [n, 8] spread like the policy's features."""
    rng = np.random.default_rng(seed)
    f = np.zeros((n, oracle.MLP_IN), dtype=np.float32)
    f[:, 0] = rng.uniform(0, 12, n)
    f[:, 1] = rng.uniform(0, 12, n)
    f[:, 2] = rng.uniform(0, 1, n)
    f[:, 3] = rng.uniform(0, 1, n) ** 3
    f[:, 4] = rng.uniform(0, 1, n) ** 3
    return oracle.bf16_array(f)


def mlp_selector_params(feature, scale=1.0):
    """logit = scale * feature_k, computed exactly: h1_0 = relu(f_k), h2_0 = relu(h1_0)."""
    H = oracle.MLP_HIDDEN
    p = np.zeros(oracle.MLP_PARAMS)
    p[oracle.P_W1 + feature * H + 0] = 1.0
    p[oracle.P_W2 + 0 * H + 0] = 1.0
    p[oracle.P_W3 + 0] = scale
    return p


def bf16_to_f64(bits):
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def load(P, g, tuning=None):
    G = P.Graph.from_host(g)
    if tuning:
        G.set_tuning(**tuning)
    return G


def step_compare(P, g, app, policy, tuning=None, stats=None, update=None, graph_obj=None, **kw):
    """Run both sides one iteration at a time; compare values every iteration
    and the edge flags after every superstep. Returns the worst PR error.

    SSSP/CC flags must be equal. PageRank flags follow the replay protocol:
    every flag that differs must belong to an edge whose oracle influence is
    within REPLAY_BAND * theta of theta; the oracle then adopts the GPU's
    flags and both continue from the same edge set. `stats` (a dict), when
    given, receives the number of such flips ("flips"), of idle iterations (a
    push from an empty frontier) and of supersteps that followed one.

    `update` (a dict: "at" = iteration after which to apply it, or None for
    when the run has ended; "batch" = (del_src, del_dst, ins_src, ins_dst,
    ins_weight); "more" = further iterations) applies one update batch to
    both sides (gg_run_update / ggo_run_update), then checks the reset
    vertices, values and flags right away and continues the comparison.
    `graph_obj`: run on this loaded graph (whose CSR must equal g's) instead
    of loading g; it is left open."""
    G = graph_obj if graph_obj is not None else load(P, g, tuning)
    sr = kw.pop("sample_ratio", 1.0)
    R = G.begin(app, sr, policy, **kw)
    okw = oracle_kw(kw)
    O = oracle.Run(g, app, policy, sigma=sr, **okw)
    assert np.array_equal(R.mask(), O.mask()) or policy == "exact", "initial sample differs"
    worst = 0.0
    flips_total = 0
    vflips_total = 0
    vs = kw.get("vstatus", "none")
    ov_prev = O.values() if vs != "none" else None
    bp_prev = (O.values(), R.values().astype(np.float64)) if app == "bp" else None
    gcur = g
    pending = dict(update) if update else None

    def apply_update():
        nonlocal gcur, bp_prev, ov_prev
        ds, dd, is_, id_, iw = pending["batch"]
        upd = oracle.apply_update(gcur, ds, dd, is_, id_, iw)
        greset = R.update(ds, dd, is_, id_, iw, more_iters=pending["more"])
        O.update(upd, more_iters=pending["more"])
        gcur = upd.graph
        oreset = O.reset_vertices()
        log("update: %d deletions, %d insertions, m %d -> %d, %d vertices reset" % (
            len(ds), len(is_), upd.deleted_old.size, gcur.m, int(oreset.sum())))
        assert np.array_equal(greset, oreset), "reset vertices differ: %d on the GPU, %d in the oracle" % (
            int(greset.sum()), int(oreset.sum()))
        if policy != "exact":
            assert np.array_equal(R.mask(), O.mask()), "edge flags differ after the update"
        gv, ov = R.values(), O.values()
        compare_values(app, gv, ov, ctx="after the update")
        if app == "bp":
            bp_prev = (ov, gv.astype(np.float64))
        if vs != "none":
            ov_prev = ov

    while True:
        if pending is not None and pending["at"] is not None and O.iterations == pending["at"]:
            apply_update()
            pending = None
        a = R.step()
        b = O.step()
        if a is None or b is None:
            assert a is None and b is None, (a, b)
            if pending is not None:
                apply_update()
                pending = None
                continue
            break
        assert a["iter"] == b.iter and a["accurate"] == b.accurate and a["superstep"] == b.superstep
        assert a["edges"] == b.edges, (a, b)
        if a.get("sparse"):
            log("iter", b.iter, "ran as a frontier push over", a["edges_processed"], "edges")
        if stats is not None:
            if a["sparse"] and a["edges_processed"] == 0:
                stats["idle"] = stats.get("idle", 0) + 1
                stats["pending"] = True
            elif a["superstep"] and stats.get("pending"):
                stats["super_after_idle"] = stats.get("super_after_idle", 0) + 1
                stats["pending"] = False
        if app in ("sssp", "cc"):
            assert a["changed"] == b.changed, (a, b)
        if a["superstep"]:
            gm, om = R.mask(), O.mask()
            flips = np.nonzero(gm != om)[0]
            if flips.size:
                infl = O.influence()
                theta = kw.get("theta0", kw.get("theta")) if b.iter == kw.get("alpha0", -2) + 1 else kw.get("theta")
                log("flips at iter", b.iter, ":", flips.size, "edges, first", flips[:5].tolist(), "oracle influence",
                    infl[flips[:5]].tolist(), "theta", theta)
                assert app in ("pr", "ppr", "bp"), "%d SSSP/CC edge flags differ after superstep %d" % (flips.size,
                                                                                                    b.iter)
                if app == "bp":
                    bad = bp_flip_justified(gcur, flips, bp_prev[0], bp_prev[1], kw.get("coupling", 0.0), theta)
                    assert not bad, "BP flag differs away from its decision band: %r" % bad[:5]
                else:
                    dist = np.abs(infl[flips] - theta)
                    assert np.all(dist <= REPLAY_BAND * theta), \
                        "flag differs away from theta: influence %r" % infl[flips[dist > REPLAY_BAND * theta][:5]].tolist()
                O.set_mask(gm)
                flips_total += int(flips.size)
            assert a["active_edges"] == int(gm.sum())
        gv = R.values()
        ov = O.values()
        if app in ("pr", "ppr", "bp"):
            worst = max(worst, rel_l1(gv, ov))
        if app == "bp":
            bp_prev = (ov, gv.astype(np.float64))
        compare_values(app, gv, ov, ctx="iter %d" % b.iter)
        if vs != "none":
            # vertex status: equal except within the band of its bound, where
            # the oracle adopts the GPU's status (replay)
            ga, oa = R.vstatus(), O.vactive()
            diff = np.nonzero(ga != oa)[0]
            if diff.size:
                eps = kw.get("eps", 0.0)
                delta = np.abs(ov - ov_prev)
                bound = eps if vs == "abs" else eps * np.abs(ov_prev)
                bound = np.broadcast_to(bound, delta.shape)
                scale = np.maximum(np.abs(ov), np.abs(ov_prev))
                far = diff[np.abs(delta[diff] - bound[diff]) > VSTATUS_BAND * scale[diff]]
                assert far.size == 0, "vertex status differs away from its bound at %s" % far[:5].tolist()
                O.set_vactive(ga)
                vflips_total += int(diff.size)
            ov_prev = ov
    log("replay: %d edge flags adopted from the GPU over the run" % flips_total)
    if vs != "none":
        log("replay: %d vertex statuses adopted from the GPU over the run" % vflips_total)
    if stats is not None:
        stats["flips"] = flips_total
        stats["vflips"] = vflips_total
    R.close()
    O.close()
    if graph_obj is None:
        G.close()
    return worst
