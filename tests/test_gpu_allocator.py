"""The library's device allocator hook (gg_set_allocator).

Every device block of a graph's workspace comes from the installed
allocator and returns to it when the graph is freed. An allocator that fails
after k successful allocations makes the call that needed the block fail
with GG_E_NOMEM, with the caller's output untouched and nothing leaked;
the same graph then completes the run once memory is available again, and
its result matches the oracle."""
import gc

import numpy as np
import pytest

import graphgen as gg
import oracle
from helpers import compare_values, device_values, graph_for, log

pytestmark = pytest.mark.gpu

NOMEM = -3
STATE = -6


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_10039_amd as P
    P.lib()
    gc.collect()
    P._close_all()  # objects left alive by earlier test modules
    assert P.live_objects() == 0
    yield P
    P.set_allocator("torch")


class Counting:
    """torch's caching allocator behind a budget of successful allocations."""

    def __init__(self, budget=1 << 30):
        import torch
        self.torch = torch
        self.held = {}
        self.budget = budget
        self.calls = 0

    def alloc(self, nbytes):
        self.calls += 1
        if self.budget <= 0:
            return 0
        self.budget -= 1
        p = self.torch.cuda.caching_allocator_alloc(nbytes)
        self.held[p] = nbytes
        return p

    def free(self, p):
        del self.held[p]
        self.torch.cuda.caching_allocator_delete(p)


def test_allocator_sees_every_block(P):
    g = graph_for("sssp", 12, 51)
    s = int(gg.pick_sources(g, 1, 51)[0])
    a = Counting()
    P.set_allocator(a.alloc, a.free)
    G = P.Graph.from_host(g)
    n_load = len(a.held)
    out, _ = G.approx_run("sssp", 0.5, "gg", alpha=3, theta=0.05, seed=2, iters=12, source=s)
    ref = oracle.run(g, "sssp", "gg", sigma=0.5, alpha=3, theta=0.05, seed=2, iters=12, source=s)
    compare_values("sssp", device_values(out, "sssp"), ref.values)
    log("blocks: %d after load, %d after a GG run, %.1f MB" % (n_load, len(a.held), sum(a.held.values()) / 1e6))
    assert n_load > 0 and len(a.held) > n_load
    with pytest.raises(P.GGError) as e:
        P.set_allocator("torch")  # a graph is alive
    assert e.value.code == STATE
    G.close()
    assert not a.held and P.live_objects() == 0
    P.set_allocator("torch")


@pytest.mark.parametrize("app", ["pr", "sssp", "cc"])
def test_allocation_failure_is_reported_and_leaks_nothing(P, app):
    import torch
    g = graph_for(app, 11, 52)
    s = int(gg.pick_sources(g, 1, 52)[0]) if app == "sssp" else 0
    it = 20 if app == "pr" else 10
    ref = oracle.run(g, app, "gg", sigma=0.5, alpha=3, theta=0.05, seed=3, iters=it, source=s)
    failures = 0
    k = 0
    while True:
        a = Counting(budget=k)
        P.set_allocator(a.alloc, a.free)
        try:
            G = P.Graph.from_host(g)
        except P.GGError as e:
            assert e.code == NOMEM, str(e)
            assert not a.held and P.live_objects() == 0, "a failed load leaked"
            failures += 1
            k += 1
            continue
        sentinel = -5 if app != "pr" else -5.0
        out = torch.full((g.n,), sentinel, dtype=P._value_dtype(app), device="cuda")
        try:
            G.approx_run(app, 0.5, "gg", out=out, alpha=3, theta=0.05, seed=3, iters=it, source=s)
            ok = True
        except P.GGError as e:
            assert e.code == NOMEM, str(e)
            torch.cuda.synchronize()
            assert bool((out == sentinel).all()), "output written by a failed run"
            failures += 1
            ok = False
        if not ok:
            # memory is back: the same graph completes the run
            a.budget = 1 << 30
            G.approx_run(app, 0.5, "gg", out=out, alpha=3, theta=0.05, seed=3, iters=it, source=s)
        compare_values(app, device_values(out, app), ref.values, ctx="budget %d" % k)
        G.close()
        assert not a.held and P.live_objects() == 0, "blocks left after the graph was freed"
        if ok:
            break
        k += 1
    P.set_allocator("torch")
    log("%s: %d allocation points failed in turn, each reported as GG_E_NOMEM" % (app, failures))
    assert failures > 3
