"""gg_exact_run_noalloc (the exact run whose per-run state lives in the
library's static per-device scratch array) against gg_exact_run on the same
graphs: PR/PPR within 1e-6 relative L1 (the same kernels in the same order,
so in practice bit for bit), SSSP/CC bit for bit. Two calls in a row share
the array, the second on a smaller graph; the first runs before the graph
has any workspace of its own. A graph whose run needs more scratch than the
array holds is rejected with GG_E_RANGE, and nothing is launched."""
import numpy as np
import pytest

import graphgen as gg
from helpers import compare_values, device_values, graph_for, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    return P


@pytest.mark.parametrize("app", ["pr", "ppr", "sssp", "cc"])
def test_noalloc_matches_exact_run(P, app):
    import torch
    for scale, seed in ((16, 41), (12, 42)):  # the second call on a smaller graph
        g = graph_for(app, scale, seed)
        src = int(gg.pick_sources(g, 1, seed)[0]) if app in ("sssp", "ppr") else 0
        log("case: noalloc", app, "scale", scale, "n", g.n, "m", g.m, "source", src)
        G = P.Graph.from_host(g)
        it = 20
        out = torch.full((g.n,), -7, dtype=P._value_dtype(app), device="cuda")
        if app in ("sssp", "cc"):
            # the exact run's iteration count, taken from a host reference
            # run of the dense iteration (max_iters large, stops at no change)
            Gx = P.Graph.from_host(g)
            it = Gx.exact_run(app, source=src)[1].iterations
            Gx.close()
        _, st = G.exact_run_noalloc(app, out, iters=it, source=src)
        torch.cuda.synchronize()
        assert st.iterations == it and st.edges_gathered == it * g.m
        want, _ = G.exact_run(app, iters=it, source=src)
        got_h = device_values(out, app)
        want_h = device_values(want, app)
        compare_values(app, got_h, want_h, ctx="noalloc %s scale %d" % (app, scale))
        if app in ("pr", "ppr"):
            log("  bitwise equal:", bool(np.array_equal(out.cpu().numpy(), want.cpu().numpy())))
        G.close()


def test_noalloc_rejects_oversized_run(P):
    """A graph with 9M vertices and no edges needs 2 x 36 MB of value
    buffers, more than the 64 MiB array: GG_E_RANGE, the output untouched."""
    import torch
    n = 9_000_000
    g = gg.Graph(n=n, rowptr=np.zeros(n + 1, dtype=np.int32), col=np.zeros(0, dtype=np.int32), weight=None,
                 name="empty_9M")
    G = P.Graph.from_host(g)
    out = torch.full((n,), 3.0, dtype=torch.float32, device="cuda")
    with pytest.raises(P.GGError) as e:
        G.exact_run_noalloc("pr", out, iters=2)
    assert e.value.code == -2  # GG_E_RANGE
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())
    G.close()


def test_noalloc_invalid_arguments(P):
    import torch
    g = graph_for("pr", 8, 43)
    G = P.Graph.from_host(g)
    out = torch.empty(g.n, dtype=torch.float32, device="cuda")
    with pytest.raises(P.GGError) as e:
        G.exact_run_noalloc("pr", out, iters=0)
    assert e.value.code == -1  # GG_E_INVAL
    with pytest.raises(P.GGError) as e:
        G.exact_run_noalloc("pr", out, damping=1.0)
    assert e.value.code == -1  # GG_E_INVAL
    with pytest.raises(P.GGError) as e:
        G.exact_run_noalloc("sssp", torch.empty(g.n, dtype=torch.int32, device="cuda"), source=1)
    assert e.value.code == -1  # GG_E_INVAL: no weights
    with pytest.raises(ValueError):
        G.exact_run_noalloc("pr", torch.empty(g.n - 1, dtype=torch.float32, device="cuda"))
    G.close()
