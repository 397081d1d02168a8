"""Shared helpers for the GPU parity tests (comparison of the HIP library
with the CPU oracle on identical seeded inputs)."""
import sys

import numpy as np

import graphgen as gg
import oracle

PR_TOL = 1e-6  # relative L1, FP32 GPU against the FP64 oracle


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
    if app in ("pr", "ppr"):
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
