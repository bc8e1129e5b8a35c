"""Serving under continuous batching (through the C ABI): each request's
result is bit-identical alone and in a mix, and equal to
zpl_bootstrap_pvalue and to the oracle; bad requests fail alone; memory
admission bounds the batches."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


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


def _datasets(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(50), np.log(20000))))
        if k % 10 == 9:
            x = (np.rint(rng.lognormal(1.0, 1.0, n)) + 1).astype(np.int64)
        else:
            x = rng.zipf(rng.uniform(1.5, 3.5), n).astype(np.int64)
        out.append(x)
    return out


def _collect(ctx, tickets, timeout_ms=60000):
    res = {}
    for t in tickets:
        r = ctx.serve_poll(t, wait_ms=timeout_ms)
        assert r is not None, "request %d did not finish" % t
        res[t] = r
    return res


def test_alone_equals_mix_equals_direct(ctx, orc):
    xs = _datasets(3, 24)
    B = 400
    ctx.serve_start()
    try:
        say("alone")
        alone = []
        for k, x in enumerate(xs[:4]):
            t = ctx.serve_submit(x, B, 1000 + k, k)
            alone.append(_collect(ctx, [t])[t])
        say("mix")
        tickets = [ctx.serve_submit(x, B, 1000 + k, k) for k, x in enumerate(xs)]
        mixed = _collect(ctx, tickets)
    finally:
        ctx.serve_stop()
    assert max(r["batch_size"] for r in mixed.values()) > 1  # requests were batched
    for k in range(4):
        a, m = alone[k], mixed[tickets[k]]
        for f in ("alpha_hat", "D", "p_value", "flags", "status"):
            assert a[f] == m[f], (k, f, a[f], m[f])
    for k, x in enumerate(xs[:6]):
        m = mixed[tickets[k]]
        d = ctx.bootstrap_pvalue(x, B, 1000 + k, k)
        assert (d["alpha_hat"], d["D"], d["p_value"]) == (m["alpha_hat"], m["D"], m["p_value"])
        o = orc.bootstrap_pvalue(x, B, 1000 + k, k)
        assert abs(o["alpha_hat"] - m["alpha_hat"]) <= 1e-10 * o["alpha_hat"]
        assert abs(o["D"] - m["D"]) < 1e-12
        assert o["p_value"] == m["p_value"]


def test_bad_request_fails_alone(ctx):
    xs = _datasets(5, 6)
    bad = np.array([1, 2, 0, 4], np.int64)
    ctx.serve_start()
    try:
        tickets = [ctx.serve_submit(x, 200, 7, k) for k, x in enumerate(xs[:3])]
        tb = ctx.serve_submit(bad, 200, 7, 99)
        tickets += [ctx.serve_submit(x, 200, 7, 10 + k) for k, x in enumerate(xs[3:])]
        res = _collect(ctx, tickets + [tb])
    finally:
        ctx.serve_stop()
    assert res[tb]["status"] == -1
    assert all(res[t]["status"] == 0 for t in tickets)


def test_memory_admission_limits_batches(ctx):
    # equal-size requests, and a budget with room for two of them but not
    # three (a request is charged 32 B per data point, 8 B per bootstrap
    # replicate and about 44 KB of table, guide and fixed scratch)
    rng = np.random.default_rng(9)
    xs = [rng.zipf(2.0, 3000).astype(np.int64) for _ in range(12)]
    B = 2000
    per = 3000 * 32 + B * 8 + 45000
    ctx.serve_start(mem_budget_bytes=2 * per + 1024)
    try:
        tickets = [ctx.serve_submit(x, B, 11, k) for k, x in enumerate(xs)]
        huge = ctx.serve_submit(np.ones(10, np.int64), 1 << 30, 1, 1)  # alone > budget
        res = _collect(ctx, tickets + [huge])
    finally:
        ctx.serve_stop()
    assert max(res[t]["batch_size"] for t in tickets) == 2
    assert all(res[t]["status"] == 0 for t in tickets)
    assert res[huge]["status"] == -2
