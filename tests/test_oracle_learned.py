"""Pins of the oracle's learned-correction pieces: bfloat16 rounding, features,
the MLP (forward, loss gradient, Adam) and the LEARNED policy's schedule.

bfloat16 rounding is checked against torch.bfloat16 over every upper half
and each rounding class of the lower half; the binary64 backward against central finite differences and torch autograd; the rounding
variant against torch with the same rounding points; Adam against
torch.optim.Adam; the policy against hand-worked examples and the special
cases that reduce it to GG or SP.
"""
import json
import os

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from helpers import bf16_to_f64, mlp_random_features, mlp_random_params, mlp_selector_params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
H, IN, NP = oracle.MLP_HIDDEN, oracle.MLP_IN, oracle.MLP_PARAMS


random_params = mlp_random_params
random_features = mlp_random_features


# --------------------------------------------------------------------------
# bfloat16
# --------------------------------------------------------------------------

def test_bf16_every_high_half_vs_torch():
    """Binary32 patterns round to the same bfloat16 as torch's conversion
    (round to nearest even; NaN compared as NaN). The rounding of a pattern
    depends on its upper 16 bits and, of the lower 16, only on how they
    compare with the halfway point 0x8000 (below, equal, above; zero or not
    for NaN payloads). So every one of the 2^16 upper halves is combined with
    lower halves that cover each class at and next to its boundaries, plus
    random ones: 2^16 x 64 patterns."""
    lows = [0x0000, 0x0001, 0x0002, 0x00FF, 0x3FFF, 0x4000, 0x7FFE, 0x7FFF, 0x8000, 0x8001, 0x8002, 0xBFFF,
            0xC000, 0xFFFE, 0xFFFF, 0x1234]
    rng = np.random.default_rng(11)
    lows += rng.integers(0, 1 << 16, 64 - len(lows)).tolist()
    hi = np.arange(1 << 16, dtype=np.uint32) << 16
    for lo in lows:
        u = hi | np.uint32(lo)
        f = u.view(np.float32)
        a = oracle.bf16_array(f)
        b = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        nan_a = ((a & 0x7F80) == 0x7F80) & ((a & 0x007F) != 0)
        nan_b = ((b & 0x7F80) == 0x7F80) & ((b & 0x007F) != 0)
        assert np.array_equal(nan_a, nan_b), hex(lo)
        ok = nan_a | (a == b)
        assert ok.all(), (hex(lo), np.nonzero(~ok)[0][:5])


def test_bf16_ties_and_specials():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even mantissa
    assert oracle.bf16_bits(1.0 + 2.0 ** -8) == 0x3F80
    assert oracle.bf16_bits(1.0 + 3 * 2.0 ** -8) == 0x3F82
    assert oracle.bf16_bits(-0.0) == 0x8000
    assert oracle.bf16_bits(float("inf")) == 0x7F80
    assert oracle.bf16_bits(3.4e38) == 0x7F80  # rounds past the largest finite bfloat16
    assert oracle.bf16_value(0x3FC0) == 1.5


# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------

def test_lg_feature_exact_at_powers_and_mitchell_bound():
    for k in range(31):
        assert oracle.lg_feature(1 << k) == float(k)
    assert oracle.lg_feature(3) == 1.5
    assert oracle.lg_feature(6) == 2.5
    ys = np.unique(np.concatenate([np.arange(1, 5000), np.random.default_rng(1).integers(1, 2**31 - 1, 4000)]))
    vals = np.array([oracle.lg_feature(int(y)) for y in ys])
    assert np.all(np.diff(vals) >= 0)
    err = np.log2(ys.astype(np.float64)) - vals
    # piecewise-linear log2 under-estimates by at most 0.0861 (maximum of
    # log2(1+t) - t on [0, 1]); binary32 rounding adds < 2^-19 relative
    assert err.min() > -1e-5 and err.max() < 0.08610


def test_delta_feature_cases():
    INF = oracle.INF
    assert oracle.delta_feature("sssp", INF, INF) == 0.0
    assert oracle.delta_feature("sssp", 7, INF) == 1.0
    assert oracle.delta_feature("sssp", 5, 10) == 0.5
    assert oracle.delta_feature("sssp", 0, 0) == 0.0
    assert oracle.delta_feature("cc", 3, 3) == 0.0
    assert oracle.delta_feature("cc", 2, 3) == 1.0

    def w(x):
        return int(np.float32(x).view(np.uint32))

    assert oracle.delta_feature("pr", w(0.5), w(0.25)) == 0.5
    assert oracle.delta_feature("pr", w(0.25), w(0.75)) == 1.0  # capped
    assert oracle.delta_feature("pr", w(0.0), w(0.25)) == 0.0
    assert oracle.delta_feature("ppr", w(0.2), w(0.2)) == 0.0


def test_features_closed_forms_star():
    """Star with every leaf pointing at the centre: the centre has in-degree
    n-1 and out-degree 0, the leaves the reverse; sigma = 1 keeps every edge."""
    g = gg.star(9)  # centre 0
    r = oracle.Run(g, "pr", "gg", sigma=1.0, alpha=2, theta=0.0, trace=True, iters=3)
    for _ in range(3):
        r.step()
    f = bf16_to_f64(r.features())
    indeg = np.diff(g.rowptr)
    outdeg = np.bincount(g.col, minlength=g.n)
    for v in range(g.n):
        assert f[v, 0] == oracle.lg_feature(1 + outdeg[v])
        assert f[v, 1] == oracle.lg_feature(1 + indeg[v])
        assert f[v, 2] == (1.0 if indeg[v] > 0 else 0.0)  # sigma = 1 keeps every edge, theta 0 too
    assert np.all(f[:, 5:] == 0)


def test_features_deltas_sssp_path():
    """Directed path 0 -> 1 -> ... -> 7 with unit weights, exact-like GG
    (sigma 1, theta 0): vertex k is reached in iteration k. At the correction
    step i (= 3, alpha = 2) delta1 compares iterations 2 and 1: 1 for vertex
    2 (newly reached), 0 elsewhere; delta2 compares iterations 1 and 0: 1 for
    vertex 1."""
    n = 8
    g = gg.from_edges(n, np.arange(n - 1), np.arange(1, n), np.ones(n - 1, dtype=np.int32))
    r = oracle.Run(g, "sssp", "gg", sigma=1.0, alpha=2, theta=0.0, trace=True, iters=3, source=0)
    for _ in range(3):
        info = r.step()
    assert info.kind == oracle.KIND_FULL
    f = bf16_to_f64(r.features())
    assert f[:, 3].tolist() == [0, 0, 1, 0, 0, 0, 0, 0]
    assert f[:, 4].tolist() == [0, 1, 0, 0, 0, 0, 0, 0]


# --------------------------------------------------------------------------
# MLP
# --------------------------------------------------------------------------

def test_mlp_backward_finite_differences():
    p = random_params(3)
    feat = random_features(4, 32)
    y = (np.random.default_rng(5).uniform(size=32) < 0.3).astype(np.float32)
    loss, grad = oracle.mlp_loss_grad(p, feat, y, pos_weight=3.0, rounding=False)
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(np.arange(oracle.P_W1, oracle.P_B1), 12, replace=False),
                          rng.choice(np.arange(oracle.P_B1, oracle.P_W2), 6, replace=False),
                          rng.choice(np.arange(oracle.P_W2, oracle.P_B2), 20, replace=False),
                          rng.choice(np.arange(oracle.P_B2, oracle.P_W3), 6, replace=False),
                          rng.choice(np.arange(oracle.P_W3, oracle.P_B3), 8, replace=False), [oracle.P_B3]])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp, _ = oracle.mlp_loss_grad(q, feat, y, 3.0, rounding=False)
        q[i] -= 2 * h
        lm, _ = oracle.mlp_loss_grad(q, feat, y, 3.0, rounding=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])) + 1e-8, (i, fd, grad[i])


def _torch_net(p, feat, rounding):
    """The same network in torch float64 autograd. With rounding, the GPU's
    rounding points are applied as straight-through roundings, and the
    gradients entering the W1/W2 products are rounded to bfloat16."""
    P = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    x = torch.tensor(bf16_to_f64(feat))

    def bf(t):  # round to bfloat16 via binary32, identity gradient
        return t + (t.to(torch.float32).to(torch.bfloat16).to(torch.float64) - t).detach()

    def f32(t):
        return t + (t.to(torch.float32).to(torch.float64) - t).detach()

    class GradBF16(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return t.clone()

        @staticmethod
        def backward(ctx, g):
            return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    W1 = P[oracle.P_W1:oracle.P_B1].view(IN, H)
    b1 = P[oracle.P_B1:oracle.P_W2]
    W2 = P[oracle.P_W2:oracle.P_B2].view(H, H)
    b2 = P[oracle.P_B2:oracle.P_W3]
    w3 = P[oracle.P_W3:oracle.P_B3]
    b3 = P[oracle.P_B3]
    if rounding:
        a1 = GradBF16.apply(x @ bf(W1))
        h1 = bf(torch.relu(f32(f32(a1) + f32(b1))))
        a2 = GradBF16.apply(h1 @ bf(W2))
        h2 = bf(torch.relu(f32(f32(a2) + f32(b2))))
        z = f32(f32(h2 @ bf(w3)) + f32(b3))
    else:
        h1 = torch.relu(x @ W1 + b1)
        h2 = torch.relu(h1 @ W2 + b2)
        z = h2 @ w3 + b3
    return P, z


@pytest.mark.parametrize("rounding", [False, True])
def test_mlp_vs_torch_autograd(rounding):
    p = random_params(7)
    feat = random_features(8, 200)
    y = (np.random.default_rng(9).uniform(size=200) < 0.2).astype(np.float32)
    pw = 4.0
    lo = oracle.mlp_forward(p, feat, rounding=rounding)
    loss, grad = oracle.mlp_loss_grad(p, feat, y, pos_weight=pw, rounding=rounding)
    P, z = _torch_net(p, feat, rounding)
    tl = torch.nn.functional.binary_cross_entropy_with_logits(
        z, torch.tensor(y, dtype=torch.float64), pos_weight=torch.tensor(pw, dtype=torch.float64))
    tl.backward()
    tol = 1e-12 if not rounding else 1e-9
    assert np.allclose(lo, z.detach().numpy(), rtol=tol, atol=tol)
    assert abs(loss - tl.item()) <= 1e-12 * max(1, abs(loss))
    tg = P.grad.numpy()
    rel = np.linalg.norm(grad - tg) / np.linalg.norm(tg)
    assert rel <= (1e-12 if not rounding else 1e-6), rel


def test_mlp_rounding_changes_little():
    """The GPU's rounding points move logits by bfloat16-sized amounts only."""
    p = random_params(11)
    feat = random_features(12, 500)
    a = oracle.mlp_forward(p, feat, rounding=False)
    b = oracle.mlp_forward(p, feat, rounding=True)
    assert np.max(np.abs(a - b) / (1 + np.abs(a))) < 0.05


def test_adam_vs_torch():
    rng = np.random.default_rng(13)
    p = rng.normal(size=300)
    m = np.zeros(300)
    v = np.zeros(300)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        g = rng.normal(size=300)
        oracle.adam_step(p, m, v, g, 3e-3, t)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------
# LEARNED policy
# --------------------------------------------------------------------------

selector_params = mlp_selector_params


def _graph_4v():
    fx = json.load(open(os.path.join(GOLDEN, "sssp_learned_4v.json")))
    e = np.array(fx["graph"]["edges_src_dst_w"])
    g = gg.from_edges(fx["graph"]["n"], e[:, 0], e[:, 1], e[:, 2].astype(np.int32))
    return fx, g


KIND_NAMES = {oracle.KIND_APPROX: "approx", oracle.KIND_ACCURATE: "accurate", oracle.KIND_FULL: "full",
              oracle.KIND_PARTIAL: "partial"}


@pytest.mark.parametrize("case", ["never_full", "full_every_2nd"])
def test_learned_golden_sssp(case):
    fx, g = _graph_4v()
    pa = fx["params"]
    c = fx["cases"][case]
    r = oracle.Run(g, "sssp", "learned", sigma=pa["sigma"], alpha=pa["alpha"], theta=pa["theta"],
                   source=pa["source"], iters=pa["iters"], mlp=selector_params(1), tau=pa["tau"], rho=pa["rho"],
                   fallback_k=c["fallback_k"])
    steps = r.run_to_end().steps
    assert [s.edges for s in steps] == c["edges_per_iteration"]
    assert [KIND_NAMES[s.kind] for s in steps] == c["kinds"]
    assert [s.selected for s in steps] == c["selected"]
    assert r.values().tolist() == c["values"]
    assert r.mask().tolist() == c["mask_after"]


def test_trace_labels_golden():
    fx, g = _graph_4v()
    t = fx["trace_labels_gg"]
    r = oracle.Run(g, "sssp", "gg", sigma=0.0, alpha=1, theta=0.5, source=0, iters=4, trace=True)
    for it in range(1, 3):
        r.step()
        lab = r.labels()
        if it == t["iteration"]:
            assert lab is not None and lab.tolist() == t["labels"]
        else:
            assert lab is None


def _compare_runs(a, b, app, check_kind=False):
    sa, sb = a.run_to_end().steps, b.run_to_end().steps
    assert [s.edges for s in sa] == [s.edges for s in sb]
    assert [s.changed for s in sa] == [s.changed for s in sb]
    if check_kind:
        assert [s.kind for s in sa] == [s.kind for s in sb]
    va, vb = a.values(), b.values()
    assert np.array_equal(va, vb)
    assert np.array_equal(a.mask(), b.mask())


CASES = [("pr", 0), ("ppr", 0), ("sssp", 0), ("cc", 0)]


def _graph(app, seed):
    if app == "cc":
        return gg.rmat(9, 8, seed=seed, symmetrize=True)
    return gg.rmat(9, 8, seed=seed, weights=True)


@pytest.mark.parametrize("app", ["pr", "ppr", "sssp", "cc"])
def test_learned_reduces_to_gg_and_sp(app):
    g = _graph(app, 21)
    src = int(gg.pick_sources(g, 1, 3)[0])
    kw = dict(sigma=0.3, alpha=3, theta=0.05, seed=4, source=src, iters=14)
    p = random_params(15)
    # fallback every correction step: GG exactly
    _compare_runs(oracle.Run(g, app, "learned", mlp=p, tau=0.0, fallback_k=1, **kw),
                  oracle.Run(g, app, "gg", **kw), app, check_kind=True)
    # everything selected (tau = -inf, rho = 1): every correction is a partial
    # superstep over all rows, i.e. GG's full superstep
    _compare_runs(oracle.Run(g, app, "learned", mlp=p, tau=-1e30, rho=1.0, **kw),
                  oracle.Run(g, app, "gg", **kw), app)
    # nothing selected, never full: the sampled graph only, i.e. SP
    _compare_runs(oracle.Run(g, app, "learned", mlp=p, tau=1e30, **kw), oracle.Run(g, app, "sp", **kw), app)


def test_learned_rho_forces_full():
    g = _graph("pr", 22)
    kw = dict(sigma=0.3, alpha=2, theta=0.05, seed=4, iters=9)
    r = oracle.Run(g, "pr", "learned", mlp=random_params(16), tau=-1e30, rho=0.5, **kw)
    steps = r.run_to_end().steps
    corr = [s for s in steps if s.iter % 3 == 0]
    assert corr and all(s.kind == oracle.KIND_FULL and s.selected == g.n for s in corr)


def _hub_share(g, min_indeg):
    indeg = np.diff(g.rowptr)
    sel = indeg >= min_indeg
    return sel.sum() / g.n, indeg[sel].sum() / g.m


def test_learned_rho_is_edge_share():
    """The fallback compares the in-edges of the selected rows with rho * m.
    The selector logit = lg(1 + in-degree) > 5 picks the rows of in-degree
    >= 32: few vertices holding a large share of the edges, so a vertex-share
    rule would take the opposite decision at both settings below."""
    g = gg.rmat(12, 16, seed=24, weights=True)
    vshare, eshare = _hub_share(g, 32)
    assert vshare < 0.15 and eshare > 0.3
    kw = dict(sigma=0.3, alpha=2, theta=0.05, seed=4, iters=6, source=0)
    for rho, want in ((eshare - 0.01, oracle.KIND_FULL), (eshare + 0.01, oracle.KIND_PARTIAL)):
        steps = oracle.Run(g, "sssp", "learned", mlp=mlp_selector_params(1), tau=5.0, rho=rho,
                           **kw).run_to_end().steps
        corr = [s for s in steps if s.iter % 3 == 0]
        assert corr and all(s.kind == want for s in corr), (rho, [s.kind for s in corr])
        assert all(s.selected == round(vshare * g.n) for s in corr)


def test_learned_partial_rows_match_their_mode():
    """Brute force on a small graph: after a partial superstep every selected
    row holds the value of an accurate update and every other row that of an
    approximate update from the same state (SSSP, integers)."""
    g = _graph("sssp", 23)
    src = int(gg.pick_sources(g, 1, 5)[0])
    p = selector_params(1)
    tau = 4.0  # lg(1 + in-degree) > 4: in-degree >= 16
    kw = dict(sigma=0.3, alpha=2, theta=0.05, seed=6, source=src, iters=6)
    r = oracle.Run(g, "sssp", "learned", mlp=p, tau=tau, **kw)
    for _ in range(2):
        r.step()
    before = r.values().astype(np.int64)
    mask = r.mask()
    info = r.step()
    assert info.kind == oracle.KIND_PARTIAL
    sel, _ = r.selection()
    after = r.values().astype(np.int64)
    INF = oracle.INF
    for u in range(g.n):
        best = before[u]
        for e in range(g.rowptr[u], g.rowptr[u + 1]):
            if not sel[u] and not mask[e]:
                continue
            xv = before[g.col[e]]
            if xv != INF:
                best = min(best, xv + int(g.weight[e]))
        assert after[u] == best, u
    indeg = np.diff(g.rowptr)
    assert np.array_equal(sel.astype(bool), indeg >= 16)


def test_learned_invalid_args():
    g = _graph("pr", 24)
    with pytest.raises(ValueError):
        oracle.Run(g, "pr", "learned")  # no network
    with pytest.raises(ValueError):
        oracle.Run(g, "pr", "learned", mlp=np.zeros(NP), fallback_k=-1)
