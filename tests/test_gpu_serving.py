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


def _stride(n):
    p2 = 1
    while p2 < n:
        p2 <<= 1
    half = max(p2, 2 * (1024 + n))
    half = (half + 1) & ~1
    return 2 * half


def test_memory_admission_limits_batches(ctx):
    # equal-size requests (n = 3,000: each fitted by a workgroup) and a budget
    # that admits two together but not a third: an active request holds 8 B
    # per bootstrap replicate + 4 KiB, and admitting k datasets of n values
    # also needs their data, 64 B each, 4 KiB and one workgroup fit's scratch
    rng = np.random.default_rng(9)
    n, B = 3000, 2000
    xs = [rng.zipf(2.0, n).astype(np.int64) for _ in range(12)]
    held = 8 * B + 4096
    fit = lambda k: k * n * 8 + k * 64 + 4096 + _stride(n) * 8  # noqa: E731
    budget = 2 * held + fit(2) + 1024
    assert budget < 3 * held + fit(3)
    ctx.serve_start(mem_budget_bytes=budget)
    try:
        tickets = [ctx.serve_submit(x, B, 11, k) for k, x in enumerate(xs)]
        huge = ctx.serve_submit(np.ones(10, np.int64), 1 << 30, 1, 1)  # alone > budget
        res = _collect(ctx, tickets + [huge])
    finally:
        ctx.serve_stop()
    assert max(res[t]["batch_size"] for t in tickets) == 2
    assert all(res[t]["status"] == 0 for t in tickets)
    assert res[huge]["status"] == -2


def test_serving_budget_above_context_budget_is_rejected():
    from paper_1305_6738_amd import Context, zpl
    with Context(0, mem_budget_bytes=1 << 30) as c:
        with pytest.raises(zpl.ZplError):
            c.serve_start(mem_budget_bytes=2 << 30)


def test_late_small_request_overlaps_and_finishes_first(ctx):
    """A short request submitted while a long bootstrap is in flight joins the
    next launch, shares it with the long one and completes before it; both
    results equal their bootstraps run alone (zpl_bootstrap_pvalue)."""
    import time
    rng = np.random.default_rng(21)
    long_x = rng.zipf(2.2, 20000).astype(np.int64)
    small_x = rng.zipf(2.7, 300).astype(np.int64)
    ctx.serve_start(slice_us=2000)
    try:
        tl = ctx.serve_submit(long_x, 1000000, 5, 1)
        time.sleep(0.01)  # the long request is admitted and its launches run
        ts = ctx.serve_submit(small_x, 500, 6, 2)
        rs = ctx.serve_poll(ts, wait_ms=60000)
        long_pending = ctx.serve_poll(tl, wait_ms=0) is None
        rl = ctx.serve_poll(tl, wait_ms=120000)
    finally:
        ctx.serve_stop()
    say("small", rs, "long", rl)
    assert rs["status"] == 0 and rl["status"] == 0
    assert long_pending, "the long bootstrap finished before the short request"
    assert rs["batch_size"] >= 2  # its launch also ran the long bootstrap's replicates
    assert rl["launches"] > rs["launches"]
    for x, B, seed, st, r in ((small_x, 500, 6, 2, rs), (long_x, 1000000, 5, 1, rl)):
        d = ctx.bootstrap_pvalue(x, B, seed, st)
        assert (d["alpha_hat"], d["D"], d["p_value"], d["flags"]) == \
            (r["alpha_hat"], r["D"], r["p_value"], r["flags"])


def test_device_datasets_equal_host_datasets(ctx):
    xs = _datasets(13, 8)
    ctx.serve_start()
    try:
        th = [ctx.serve_submit(x, 300, 40 + k, k) for k, x in enumerate(xs)]
        td = [ctx.serve_submit(torch.from_numpy(x).cuda(), 300, 40 + k, k)
              for k, x in enumerate(xs)]
        res = _collect(ctx, th + td)
    finally:
        ctx.serve_stop()
    for a, b in zip(th, td):
        for f in ("status", "alpha_hat", "D", "p_value", "flags"):
            assert res[a][f] == res[b][f], f


def test_one_large_dataset_among_many_small_ones(ctx):
    """A dataset of two million values admitted beside 255 small ones: the
    batched fit's scratch is charged as it is allocated, and every request
    completes (none fails the scheduler)."""
    rng = np.random.default_rng(17)
    big = rng.zipf(2.0, 2_000_000).astype(np.int64)
    smalls = [rng.zipf(2.5, 100).astype(np.int64) for _ in range(255)]
    ctx.serve_start(mem_budget_bytes=256 << 20)
    try:
        tickets = [ctx.serve_submit(big, 200, 3, 0)]
        tickets += [ctx.serve_submit(x, 200, 3, 1 + k) for k, x in enumerate(smalls)]
        res = _collect(ctx, tickets)
    finally:
        ctx.serve_stop()
    assert all(r["status"] == 0 for r in res.values()), \
        sorted(set(r["status"] for r in res.values()))
    d = ctx.bootstrap_pvalue(big, 200, 3, 0)
    r = res[tickets[0]]
    assert (d["alpha_hat"], d["D"], d["p_value"]) == (r["alpha_hat"], r["D"], r["p_value"])
