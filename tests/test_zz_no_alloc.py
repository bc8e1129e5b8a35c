"""The allocation-free fit (zpl_fit_noalloc): same results as zpl_fit and
zpl_fit_truncated, through the C ABI, on two calls in a row (the second on a
smaller dataset, so stale scratch from the first would show)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1305_6738_amd import Context
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with Context(0) as c:
        yield c


def _dataset(alpha, n, seed, kmax=0):
    import torch
    x = np.random.Generator(np.random.PCG64(seed)).zipf(alpha, size=n)
    if kmax:
        x = np.minimum(x, kmax)
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int64)).cuda()


def _noalloc(ctx, x, kmax=0):
    import torch
    a = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    D = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    f = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    ctx.fit_noalloc(x, a, D, f, st, kmax=kmax)
    torch.cuda.synchronize()
    return float(a.item()), float(D.item()), int(f.item()) & 0xffffffff, int(st.item())


@pytest.mark.parametrize("kmax", [0, 1000])
def test_noalloc_matches_fit_on_two_calls(ctx, kmax):
    for alpha, n, seed in ((1.6, 300000, 5), (2.5, 1500, 6)):  # second call smaller
        x = _dataset(alpha, n, seed, kmax)
        a, D, f, st = _noalloc(ctx, x, kmax)
        ref = ctx.fit(x, kmax=kmax)
        print("noalloc kmax=%d n=%d: %r vs %r" % (kmax, n, (a, D, f, st), ref), flush=True)
        assert st == 0
        assert f == ref["flags"]
        assert abs(a - ref["alpha_hat"]) <= 1e-10 * max(abs(ref["alpha_hat"]), 1.0)
        assert abs(D - ref["D"]) <= 1e-12
        assert (a, D) == (ref["alpha_hat"], ref["D"])  # same kernel arithmetic: same bits


def test_noalloc_edge_cases(ctx):
    import torch
    from paper_1305_6738_amd import zpl
    one = torch.ones(1, dtype=torch.int64, device="cuda")
    a, D, f, st = _noalloc(ctx, one)
    ref = ctx.fit(one)
    assert st == 0 and (a, D, f) == (ref["alpha_hat"], ref["D"], ref["flags"])
    bad = torch.tensor([3, 0, 2], dtype=torch.int64, device="cuda")
    assert _noalloc(ctx, bad)[3] == 2
    above = torch.tensor([3, 21, 2], dtype=torch.int64, device="cuda")
    assert _noalloc(ctx, above, kmax=20)[3] == 2
    big = torch.ones((1 << 20) + 1, dtype=torch.int64, device="cuda")
    out = [torch.zeros(1, dtype=t, device="cuda")
           for t in (torch.float64, torch.float64, torch.int32, torch.int32)]
    with pytest.raises(zpl.ZplError):
        ctx.fit_noalloc(big, *out)
    full = _dataset(1.8, 1 << 20, 9)
    a, D, f, st = _noalloc(ctx, full)
    ref = ctx.fit(full)
    assert st == 0 and (a, D, f) == (ref["alpha_hat"], ref["D"], ref["flags"])
