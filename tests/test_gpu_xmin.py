"""GPU parity of the law with a lower cutoff xmin (p(k) = k^-alpha /
zeta(alpha, xmin), k >= xmin), of fitting the values >= xmin of a dataset
and of the KS-minimising choice of xmin, against the oracle through the C ABI.

Bar (the same as the pure law's): draws and per-replicate multiset
fingerprints bit-exact; alpha_hat within 1e-10 relative; D within 1e-12;
quantiles equal to the oracle's order statistic of the GPU's D array; the
chosen candidate equal to the oracle's unless the two smallest D lie within
the D tolerance of each other.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

QS = [(9, 10), (95, 100), (99, 100), (999, 1000)]
KEEP_FLAGS = 1 | 2 | 8  # ALL_ONES, TAIL_CAPPED, NOCONV


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
    alpha, n, R, seed, stream, _, xmin = cell
    if reps is None:
        ref = orc.hz_simulate(alpha, xmin, n, seed, stream, 0, R)
        idx = np.arange(R)
    else:
        idx = np.asarray(sorted(set(int(r) for r in reps)))
        parts = [orc.hz_simulate(alpha, xmin, n, seed, stream, int(r), 1) for r in idx]
        ref = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    gi = lo + idx
    assert np.array_equal(g["fp"][gi], ref["fp"]), cell
    assert np.array_equal(g["flags"][gi] & KEEP_FLAGS, ref["flags"] & KEEP_FLAGS), cell
    assert np.all(np.abs(g["alpha_hat"][gi] - ref["alpha_hat"]) <= 1e-10 * ref["alpha_hat"]), cell
    assert np.all(np.abs(g["D"][gi] - ref["D"]) <= 1e-12), cell


@pytest.mark.parametrize("a,xmin", [(2.5, 2), (1.6, 17), (3.3, 18), (2.0, 500), (1.8, 123456),
                                    (30.0, 17), (50.0, 20), (12.0, 16),
                                    # xmin^-a below FP64's range: sums relative to xmin^-a
                                    (30.0, 10**6), (2.5, 2**40), (64.0, 10**9), (12.0, 4097)])
def test_cdf_table_matches_oracle(ctx, orc, a, xmin):
    T = torch.zeros(4096, dtype=torch.float64, device="cuda")
    ctx.cdf_table(a, T, xmin=xmin)
    torch.cuda.synchronize()
    ref = orc.hz_cdf_table(a, xmin)
    assert np.abs(T.cpu().numpy() - ref).max() <= 4e-15, (a, xmin)


@pytest.mark.parametrize("a,xmin,n", [(2.5, 3, 1001), (1.6, 500, 600), (4.0, 2, 257),
                                      (1.3, 40, 300), (2.2, 100000, 129), (30.0, 10**9, 200)])
def test_draws_bit_exact(ctx, orc, a, xmin, n):
    count = 5
    say("draws", a, xmin, n)
    x = torch.zeros(count * n, dtype=torch.int64, device="cuda")
    f = torch.zeros(count, dtype=torch.int32, device="cuda")
    ctx.sample_draws(a, n, 7, 2, 13, count, x, f, xmin=xmin)
    torch.cuda.synchronize()
    got = x.cpu().numpy().reshape(count, n)
    fl = f.cpu().numpy().view(np.uint32)
    for r in range(count):
        want, wf = orc.hz_sample(a, xmin, n, 7, 2, 13 + r)
        assert np.array_equal(got[r], want), (a, xmin, r)
        assert (fl[r] & 2) == (wf & 2)


CELLS = [
    (2.5, 100, 700, 42, 0, 0, 2),
    (1.6, 300, 200, 42, 1, 0, 17),        # heavy tail: many draws past xmin + 4096
    (4.0, 3, 513, 7, 2, 0, 2),            # about 44 % of replicates all at the cutoff
    (2.2, 1000, 130, 9, 3, 0, 1000),      # every value above the LDS histogram
    (60.0, 20, 300, 9, 4, 0, 300),        # exponent near the bracket end: some NOCONV
    (3.0, 57, 64, 1, 5, 0, 5),
]


def test_simulate_cells_match_oracle(ctx, orc):
    say("simulate cutoff cells")
    g = run_cells(ctx, CELLS)
    lo = 0
    for ci, cell in enumerate(CELLS):
        compare(orc, g, lo, cell)
        D = g["D"][lo:lo + cell[2]]
        for qi, (a, b) in enumerate(QS):
            assert g["q"][ci, qi] == orc.quantile(D, a, b), (cell, (a, b))
        lo += cell[2]
    # the all-at-cutoff rule and the bracket end are exercised
    assert np.any(g["flags"][700 + 200:700 + 200 + 513] & 1)
    assert np.any(g["flags"][700 + 200 + 513 + 130:700 + 200 + 513 + 130 + 300] & 8)


def test_large_exponents_at_small_cutoffs(ctx, orc):
    """Exponents far above 2 with cutoffs near 17: zeta(a, q) is then the
    whole normaliser, and its Euler-Maclaurin tail must start at 1.6 a + 10
    (at q = 17 it is off by 4e-15 at a = 10 and 2e-4 at a = 64).  Every
    replicate against the oracle, and fits of data piled at the cutoff."""
    cells = [(25.0, 50, 400, 5, 10, 0, 17), (12.0, 200, 300, 5, 11, 0, 3),
             (40.0, 30, 300, 5, 12, 0, 20), (9.0, 100, 300, 5, 13, 0, 16),
             (60.0, 40, 200, 5, 14, 0, 30)]
    say("large exponents at small cutoffs")
    g = run_cells(ctx, cells)
    lo = 0
    for cell in cells:
        compare(orc, g, lo, cell)
        lo += cell[2]
    for xmin in (2, 16, 17, 20):
        for extra in ([1, 1, 1], [1, 1, 2], [1] * 6 + [3]):
            x = np.array([xmin] * 60 + [xmin + e for e in extra])
            r = ctx.fit(x, xmin=xmin)
            ref = orc.hz_fit(x, xmin)
            assert abs(r["alpha_hat"] - ref["alpha_hat"]) <= 1e-10 * ref["alpha_hat"], (xmin, extra)
            assert abs(r["D"] - ref["D"]) <= 1e-12, (xmin, extra)
            s = ctx.fit_scan(x, [xmin])
            assert (s["alpha_hat"][0], s["D"][0]) == (r["alpha_hat"], r["D"])


HUGE = [(2.5, 200, 300, 5, 20, 0, 10**6), (30.0, 100, 200, 5, 21, 0, 10**9),
        (1.5, 100, 200, 5, 22, 0, 2**40), (64.0, 50, 200, 5, 23, 0, 70000),
        (27.0, 150, 200, 5, 24, 0, 2**33)]


def test_huge_cutoffs(ctx, orc):
    """Cutoffs where xmin^-a is below FP64's range (a ln xmin > 708), up to the
    2^40 limit: the Hurwitz sums of eq. 2 and the CDF of eq. 1 are taken
    relative to xmin^-a.  Every replicate against the oracle, the quantiles,
    no bracket-end NOCONV where the exponent is far from 64, and fits of data
    with a body below the cutoff (single fit and scan candidate agree bit for
    bit)."""
    say("huge cutoffs: cells")
    g = run_cells(ctx, HUGE)
    lo = 0
    for ci, cell in enumerate(HUGE):
        compare(orc, g, lo, cell)
        D = g["D"][lo:lo + cell[2]]
        for qi, (a, b) in enumerate(QS):
            assert g["q"][ci, qi] == orc.quantile(D, a, b), (cell, (a, b))
        if cell[0] < 60.0:
            assert not np.any(g["flags"][lo:lo + cell[2]] & 8), cell
        lo += cell[2]
    say("huge cutoffs: fits")
    for a, xmin in [(2.5, 10**6), (30.0, 10**9), (40.0, 2**40), (3.0, 4097), (64.0, 10**5)]:
        tail, _ = orc.hz_sample(a, xmin, 2000, 9, 0, 0)
        body = np.random.default_rng(xmin % 1000).integers(1, xmin, size=500)
        x = np.concatenate([body, tail])
        r = ctx.fit(x, xmin=xmin)
        ref = orc.hz_fit(x, xmin)
        assert ref["flags"] & 8 == 0 and r["flags"] & KEEP_FLAGS == ref["flags"] & KEEP_FLAGS
        assert abs(r["alpha_hat"] - ref["alpha_hat"]) <= 1e-10 * ref["alpha_hat"], (a, xmin)
        assert abs(r["D"] - ref["D"]) <= 1e-12, (a, xmin)
        assert r["n_tail"] == ref["n_tail"] == 2000
        s = ctx.fit_scan(x, [xmin])
        assert (s["alpha_hat"][0], s["D"][0]) == (r["alpha_hat"], r["D"])


def test_cutoff_cells_beside_pure_cells_bit_identical(ctx):
    pure = [(2.5, 100, 400, 1, 0, 0, 0), (1.75, 50, 300, 1, 1, 0, 1)]
    cut = [(2.5, 100, 400, 1, 2, 0, 10), (1.5, 40, 300, 1, 3, 0, 3)]
    a = run_cells(ctx, pure)
    b = run_cells(ctx, cut)
    m = run_cells(ctx, [pure[0], cut[0], pure[1], cut[1]])
    assert np.array_equal(m["D"][:400], a["D"][:400])
    assert np.array_equal(m["D"][400:800], b["D"][:400])
    assert np.array_equal(m["D"][800:1100], a["D"][400:])
    assert np.array_equal(m["D"][1100:], b["D"][400:])
    # xmin = 0 and xmin = 1 are the pure law
    assert np.array_equal(a["fp"][400:], run_cells(ctx, [pure[1][:6] + (0,)])["fp"])


def test_full_size_cell_sampled(ctx, orc):
    """n = 10,000, R = 20,000 at xmin = 10 in the batched launch; sampled
    replicates recomputed by the oracle."""
    cell = (2.5, 10000, 20000, 42, 9, 0, 10)
    say("full-size cutoff cell")
    g = run_cells(ctx, [cell])
    rng = np.random.default_rng(3)
    compare(orc, g, 0, cell, reps=[0, 19999] + list(rng.integers(0, 20000, 12)))
    for qi, (a, b) in enumerate(QS):
        assert g["q"][0, qi] == orc.quantile(g["D"], a, b)


def _mixture(orc, seed, n_body, n_tail, x0, a):
    rng = np.random.default_rng(seed)
    body = rng.integers(1, x0, size=n_body)
    tail, _ = orc.hz_sample(a, x0, n_tail, seed, 0, 0)
    return np.concatenate([body, tail])


@pytest.mark.parametrize("xmin", [1, 2, 9, 17, 18, 60, 1500])
def test_fit_xmin_matches_oracle(ctx, orc, xmin):
    x = _mixture(orc, 5, 3000, 4000, 60, 2.3)
    r = ctx.fit(x, xmin=xmin)
    ref = orc.hz_fit(x, xmin)
    assert abs(r["alpha_hat"] - ref["alpha_hat"]) <= 1e-10 * ref["alpha_hat"]
    assert abs(r["D"] - ref["D"]) <= 1e-12
    assert r["flags"] & KEEP_FLAGS == ref["flags"] & KEEP_FLAGS
    if xmin > 1:
        assert r["n_tail"] == ref["n_tail"]
    # device input gives the same result
    rd = ctx.fit(torch.from_numpy(x).cuda(), xmin=xmin)
    assert (rd["alpha_hat"], rd["D"]) == (r["alpha_hat"], r["D"])
    # the scan's candidate runs the same arithmetic as the single fit (at
    # xmin = 1 the pure law's: the workgroup fit of zpl_fit, bit for bit)
    s = ctx.fit_scan(x, [xmin])
    assert (s["alpha_hat"][0], s["D"][0]) == (r["alpha_hat"], r["D"])


def test_fit_xmin_edge_cases(ctx, orc):
    from paper_1305_6738_amd import ZplError
    for x, xmin in [(np.full(9, 7), 7), (np.array([300] * 12 + [301, 303]), 300),
                    (np.array([5, 5, 6]), 5), (np.array([2, 40, 41, 300, 3]), 3)]:
        r = ctx.fit(x, xmin=xmin)
        ref = orc.hz_fit(x, xmin)
        assert r["flags"] & KEEP_FLAGS == ref["flags"] & KEEP_FLAGS, (x, xmin)
        assert abs(r["alpha_hat"] - ref["alpha_hat"]) <= 1e-10 * ref["alpha_hat"], (x, xmin)
        assert abs(r["D"] - ref["D"]) <= 1e-12, (x, xmin)
    with pytest.raises(ZplError):
        ctx.fit(np.array([1, 2, 3]), xmin=4)  # no value at or above the cutoff
    with pytest.raises(ZplError):
        ctx.fit(np.array([0, 5, 6]), xmin=5)  # a value below 1


def test_fit_scan_matches_oracle(ctx, orc):
    x = _mixture(orc, 11, 2500, 5000, 40, 2.6)
    cand = np.concatenate([np.arange(1, 151), [400, 10 ** 9]])
    say("scan", len(cand), "candidates on", x.size, "values")
    g = ctx.fit_scan(x, cand)
    r = orc.hz_scan(x, cand)
    assert np.array_equal(g["n_tail"], r["n_tail"])
    fin = np.isfinite(r["D"])
    assert np.array_equal(np.isfinite(g["D"]), fin)
    assert np.all(np.abs(g["D"][fin] - r["D"][fin]) <= 1e-12)
    assert np.all(np.abs(g["alpha_hat"][fin] - r["alpha_hat"][fin]) <= 1e-10 * r["alpha_hat"][fin])
    assert np.array_equal(g["flags"] & KEEP_FLAGS, r["flags"] & KEEP_FLAGS)
    d = np.sort(r["D"][fin])
    if d[1] - d[0] > 2e-12:
        assert g["best"] == r["best"]
    else:
        assert g["D"][g["best"]] <= d[0] + 1e-12
    assert 30 <= cand[g["best"]] <= 55


def test_invalid_cutoff_arguments(ctx):
    from paper_1305_6738_amd import ZplError
    bad = [dict(cells=[(2.5, 10, 10, 1, 0, 20, 5)]),           # xmin with the truncated law
           dict(cells=[(2.5, 10, 10, 1, 0, 0, -3)]),
           dict(cells=[(2.5, 10, 10, 1, 0, 0, 2 ** 41)]),
           dict(cells=[(2.5, 10, 10, 1, 0, 0, 5)], form="lane"),
           dict(cells=[(2.5, 10, 10, 1, 0, 0, 5)], form="wave")]
    for kw in bad:
        with pytest.raises(ZplError) as e:
            ctx.simulate_cells(**kw)
        assert e.value.status == -1, kw
    with pytest.raises(ZplError):
        ctx.fit_scan(np.array([1, 2, 3]), [0])
    with pytest.raises(ZplError):
        ctx.fit_scan(np.array([1, 0, 3]), [1, 2])
    r = ctx.fit_scan(np.array([1, 2, 3]), [5, 9])
    assert r["best"] == -1 and np.all(np.isinf(r["D"]))
