"""Autotuner on the GPU, and plan-buffer reuse by hipGraph replays.

Every execution form gives the same bits, so a tuned plan must reproduce the
untuned outputs exactly; the measured table must cover exactly the eligible
(point, form) pairs.  A graph replay after other calls have rewritten the
context's plan buffers must still simulate its own cells.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

QS = [(9, 10), (95, 100), (99, 100)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_6738_amd import Context
    c = Context(0)
    yield c
    c.close()


def outputs(ctx, cells, **kw):
    R = sum(c[2] for c in cells)
    d = torch.zeros(R, dtype=torch.float64, device="cuda")
    a = torch.zeros(R, dtype=torch.float64, device="cuda")
    fp = torch.zeros(R, dtype=torch.int64, device="cuda")
    q = ctx.simulate_cells(cells, quantiles=QS, d_out=d, alpha_hat_out=a, fingerprint_out=fp, **kw)
    torch.cuda.synchronize()
    return q, d.cpu().numpy(), a.cpu().numpy(), fp.cpu().numpy()


def same(x, y):
    return all(np.array_equal(u, v) for u, v in zip(x, y))


def test_autotune_table_shape_and_eligibility(ctx):
    from paper_1305_6738_amd import plan_forms
    alphas, ns = [1.5, 2.5, 3.5], [10, 300, 10000]
    say("autotune", alphas, ns)
    t = ctx.autotune(alphas, ns)
    assert [(e["alpha"], e["n"]) for e in t] == [(a, n) for a in alphas for n in ns]
    for e in t:
        c = e["ns_per_replicate"]
        assert c[2] > 0.0, e  # the heavy form is always measured
        for f in range(3):
            assert c[f] == -1.0 or c[f] > 0.0, e
    # the lane form is eligible at small n with light tails, not at (1.5, 1e4)
    by = {(e["alpha"], e["n"]): e["ns_per_replicate"] for e in t}
    assert by[(3.5, 10)][0] > 0 and by[(1.5, 10000)][0] == -1.0
    # for a cell of many replicates the planner picks the cheapest measured
    # form at a grid point
    for (a, n), c in by.items():
        best = min((v, f) for f, v in enumerate(c) if v > 0)[1]
        assert plan_forms([(a, n, 10 ** 6, 1, 0)], t) == [["lane", "wave", "heavy"][best]]
    ctx.set_tuning(None)


def test_tuned_plan_bit_identical(ctx):
    from paper_1305_6738_amd import plan_forms
    from inputs import uneven_cells
    cells = [c[:2] + (300,) + c[3:] for c in uneven_cells(count=48, R=300, seed=5)]
    cells = [c for c in cells if c[1] <= 20000]
    say("untuned", len(cells), "cells")
    ctx.set_tuning(None)
    base = outputs(ctx, cells)
    # tables that force each form where eligible
    for f, name in enumerate(["lane", "wave", "heavy"]):
        cost = [5.0, 5.0, 5.0]
        cost[f] = 1.0
        t = [{"alpha": a, "n": n, "ns_per_replicate": cost} for a in (1.5, 3.5)
             for n in (10, 100000)]
        say("tuned toward", name, plan_forms(cells, t).count(name), "cells")
        ctx.set_tuning(t)
        assert same(outputs(ctx, cells), base), name
    ctx.set_tuning(None)


def test_graph_replay_after_other_calls(ctx):
    A = [(2.5, 200, 700, 11, 0), (1.75, 60, 513, 11, 1)]
    B = [(3.0, 50, 900, 12, 0)]
    say("graph replay with interleaved calls")
    eager_a = outputs(ctx, A)
    g1 = outputs(ctx, A, use_graph=True)  # capture
    assert same(g1, eager_a)
    eager_b = outputs(ctx, B)  # rewrites the plan buffers
    assert same(outputs(ctx, A, use_graph=True), eager_a)  # replay must re-upload A's plan
    x = np.arange(1, 51, dtype=np.int64)
    ctx.bootstrap_pvalue(x, 300, seed=3)  # another writer of the plan buffers
    T = torch.zeros(4096, dtype=torch.float64, device="cuda")
    ctx.cdf_table(2.0, T)
    for _ in range(3):
        assert same(outputs(ctx, A, use_graph=True), eager_a)
    assert same(outputs(ctx, B), eager_b)


def test_graph_replay_after_tuning_change(ctx):
    """A captured graph is tied to its plan: after the tuning table changes
    the forms (and so the units), the next graph call must capture anew."""
    from paper_1305_6738_amd import plan_forms
    A = [(2.5, 200, 100000, 21, 0), (3.0, 60, 50000, 21, 1)]
    ctx.set_tuning(None)
    eager = outputs(ctx, A)
    for f, name in [(0, "lane"), (2, "heavy"), (1, "wave")]:
        cost = [5.0, 5.0, 5.0]
        cost[f] = 1.0
        t = [{"alpha": a, "n": n, "ns_per_replicate": cost} for a in (1.5, 3.5)
             for n in (10, 100000)]
        ctx.set_tuning(t)
        forms = plan_forms(A, t)
        say("graph under tuning toward", name, forms)
        assert forms == [name, name]
        assert same(outputs(ctx, A, use_graph=True), eager), name
        assert same(outputs(ctx, A, use_graph=True), eager), name  # replay
    ctx.set_tuning(None)
