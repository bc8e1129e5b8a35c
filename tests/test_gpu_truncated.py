"""GPU parity of the truncated law on 1..K (Sect. 1 with a finite upper
limit; Tables 2-6) against the oracle, through the C ABI.

Bar: draws and histogram fingerprints bit-exact; alpha_hat within
1e-10 * max(|alpha_hat|, 1) (the truncated law's exponent can be 0, where a
purely relative tolerance has no meaning); D within 1e-12; quantiles equal to
the oracle's order statistic of the GPU's D array.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

QS = [(9, 10), (95, 100), (99, 100), (999, 1000)]


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


def run_cells(ctx, cells, **kw):
    R = sum(c[2] for c in cells)
    d = torch.zeros(R, dtype=torch.float64, device="cuda")
    a = torch.zeros(R, dtype=torch.float64, device="cuda")
    f = torch.zeros(R, dtype=torch.int32, device="cuda")
    fp = torch.zeros(R, dtype=torch.int64, device="cuda")
    q = ctx.simulate_cells(cells, quantiles=QS, d_out=d, alpha_hat_out=a, flags_out=f,
                           fingerprint_out=fp, **kw)
    torch.cuda.synchronize()
    return {"q": q, "D": d.cpu().numpy(), "alpha_hat": a.cpu().numpy(),
            "flags": f.cpu().numpy().view(np.uint32), "fp": fp.cpu().numpy().view(np.uint64)}


def compare(orc, g, lo, cell, reps=None):
    alpha, n, R, seed, stream, K = cell
    if reps is None:
        ref = orc.tz_simulate(alpha, K, n, seed, stream, 0, R)
        idx = np.arange(R)
    else:
        idx = np.asarray(sorted(set(int(r) for r in reps)))
        parts = [orc.tz_simulate(alpha, K, n, seed, stream, int(r), 1) for r in idx]
        ref = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    gi = lo + idx
    assert np.array_equal(g["fp"][gi], ref["fp"]), cell
    assert np.array_equal(g["flags"][gi] & 9, ref["flags"] & 9), cell  # ALL_ONES, NOCONV
    da = np.abs(g["alpha_hat"][gi] - ref["alpha_hat"])
    assert (da <= 1e-10 * np.maximum(np.abs(ref["alpha_hat"]), 1.0)).all(), (cell, da.max())
    assert np.abs(g["D"][gi] - ref["D"]).max() <= 1e-12, cell


def test_table_matches_oracle(ctx, orc):
    for g, K in [(0.25, 20), (1.0, 50), (2.5, 1000), (-0.5, 100), (1.0, 4096)]:
        say("table", g, K)
        T = torch.zeros(4096, dtype=torch.float64, device="cuda")
        ctx.cdf_table(g, T, kmax=K)
        torch.cuda.synchronize()
        t = T.cpu().numpy()
        ref = orc.tz_cdf_table(g, K)
        assert np.abs(t[:K] - ref).max() <= K * 2.0 ** -52, (g, K)
        assert (t[K - 1:] == 1.0).all()


@pytest.mark.parametrize("g,K,n", [(0.25, 20, 1001), (1.0, 100, 300), (3.5, 1000, 64),
                                   (-0.3, 50, 257), (0.75, 4096, 500)])
def test_draws_bit_exact(ctx, orc, g, K, n):
    count = 7
    say("draws", g, K, n)
    x = torch.zeros(count * n, dtype=torch.int64, device="cuda")
    f = torch.zeros(count, dtype=torch.int32, device="cuda")
    ctx.sample_draws(g, n, 5, 3, 11, count, x, f, kmax=K)
    torch.cuda.synchronize()
    got = x.cpu().numpy().reshape(count, n)
    for r in range(count):
        assert np.array_equal(got[r], orc.tz_sample(g, K, n, 5, 3, 11 + r)), (g, K, r)


@pytest.mark.parametrize("form", ["auto", "lane", "wave", "heavy"])
def test_simulate_all_forms(ctx, orc, form):
    cells = [(0.25, 100, 300, 42, 0, 20), (1.0, 37, 200, 42, 1, 50), (2.5, 10, 520, 7, 2, 20),
             (4.0, 10, 300, 7, 3, 1000), (1.5, 300, 130, 9, 4, 500), (-0.2, 60, 70, 9, 5, 100),
             # spread over a large support: most draws take the deferred path
             (0.5, 150, 130, 9, 6, 1000), (0.0, 40, 90, 3, 7, 2000)]
    say("simulate truncated", form)
    g = run_cells(ctx, cells, form=form)
    lo = 0
    for ci, cell in enumerate(cells):
        compare(orc, g, lo, cell)
        D = g["D"][lo:lo + cell[2]]
        for qi, (a, b) in enumerate(QS):
            assert g["q"][ci, qi] == orc.quantile(D, a, b)
        lo += cell[2]


@pytest.mark.parametrize("form", ["auto", "wave", "heavy"])
def test_no_root_at_small_K(ctx, orc, form):
    """K = 2 and 3 with small samples: a replicate whose values all equal K
    has no root (mu < ln K everywhere, and for K = 2 mu reaches ln K to FP64
    rounding near s = -53).  Like the oracle, the GPU returns the bracket end
    -64 with NOCONV for every such replicate, in every form."""
    cells = [(0.25, 5, 3000, 3, 0, 2), (-1.0, 5, 2000, 3, 1, 2), (-2.0, 4, 2000, 3, 2, 3)]
    say("no root at small K", form)
    g = run_cells(ctx, cells, form=form)
    lo = 0
    for cell in cells:
        compare(orc, g, lo, cell)
        lo += cell[2]
    edge = g["alpha_hat"] == -64.0
    assert edge.sum() > 100 and np.all(g["flags"][edge] & 8)
    r = ctx.fit(np.full(7, 2, dtype=np.int64), kmax=2)
    assert r["status"] == -4 and r["alpha_hat"] == -64.0


def test_large_support_in_the_heavy_form(ctx, orc):
    """K = 3000 and 4096 with exponents at or below 0.25: most values lie
    above the heavy form's 1,024-bin histogram, so the overflow (thousands
    of values) takes the global sort before the K-term finish.  Every
    replicate against the oracle."""
    cells = [(0.25, 3000, 40, 5, 60, 4096), (0.0, 5000, 30, 5, 61, 4096),
             (-0.5, 2000, 30, 5, 62, 3000)]
    from paper_1305_6738_amd import plan_forms
    assert plan_forms(cells) == ["heavy"] * 3
    say("large support, heavy form")
    g = run_cells(ctx, cells)
    lo = 0
    for cell in cells:
        compare(orc, g, lo, cell)
        lo += cell[2]


def test_mixed_with_pure_cells_bit_identical(ctx):
    pure = [(2.5, 100, 400, 1, 0, 0), (1.75, 50, 300, 1, 1, 0)]
    trunc = [(1.0, 100, 400, 1, 2, 20), (0.5, 200, 300, 1, 3, 1000)]
    say("mixed laws")
    a = run_cells(ctx, pure)
    b = run_cells(ctx, trunc)
    m = run_cells(ctx, [pure[0], trunc[0], pure[1], trunc[1]])
    assert np.array_equal(m["D"][:400], a["D"][:400])
    assert np.array_equal(m["D"][400:800], b["D"][:400])
    assert np.array_equal(m["D"][800:1100], a["D"][400:])
    assert np.array_equal(m["D"][1100:], b["D"][400:])


def test_table2_slice_sampled(ctx, orc):
    """K = 20, the 12 exponents of Table 2 at N = 100, R = 50,000 in one
    batched launch: sampled replicates vs the oracle, quantiles by the
    oracle's rule on the GPU's D."""
    gammas = [0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 3.5, 4.0]
    cells = [(g, 100, 50000, 42, i, 20) for i, g in enumerate(gammas)]
    say("Table 2 slice")
    g = run_cells(ctx, cells)
    rng = np.random.default_rng(5)
    lo = 0
    for ci, cell in enumerate(cells):
        compare(orc, g, lo, cell, list(rng.integers(0, cell[2], 20)) + [0, cell[2] - 1])
        D = g["D"][lo:lo + cell[2]]
        for qi, (a, b) in enumerate(QS):
            assert g["q"][ci, qi] == orc.quantile(D, a, b)
        lo += cell[2]


def test_fit_truncated(ctx, orc):
    from paper_1305_6738_amd import ZplError
    rng = np.random.default_rng(4)
    for K in (2, 20, 1000, 4096):
        for _ in range(3):
            x = np.minimum(rng.zipf(1.3, size=int(rng.integers(5, 3000))), K).astype(np.int64)
            r = ctx.fit(x, kmax=K)
            ref = orc.tz_fit(x, K)
            assert abs(r["alpha_hat"] - ref["alpha_hat"]) <= 1e-10 * max(abs(ref["alpha_hat"]), 1)
            assert abs(r["D"] - ref["D"]) <= 1e-12
    r = ctx.fit(np.arange(1, 21, dtype=np.int64), kmax=20)  # uniform: g_hat = 0
    assert abs(r["alpha_hat"]) < 1e-12 and r["D"] < 1e-14
    r = ctx.fit(np.full(9, 20, dtype=np.int64), kmax=20)  # no root in [-64, 64]
    assert r["status"] == -4 and r["alpha_hat"] == -64.0
    with pytest.raises(ZplError):
        ctx.fit(np.array([1, 21], dtype=np.int64), kmax=20)
    with pytest.raises(ZplError):
        ctx.fit(np.array([1, 2], dtype=np.int64), kmax=4097)
