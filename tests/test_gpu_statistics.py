"""Statistical behaviour of the bespoke test the paper recommends (Sect. 4):
under the null hypothesis (data drawn from the discrete power law at some
exponent, the exponent then estimated), the parametric-bootstrap p-value is
close to uniform on (0, 1); against data from another law it is small."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_6738_amd import Context
    c = Context(0)
    yield c
    c.close()


def _draws(ctx, alpha, n, seed, stream_id):
    x = torch.zeros(n, dtype=torch.int64, device="cuda")
    f = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.sample_draws(alpha, n, seed, stream_id, 0, 1, x, f)
    torch.cuda.synchronize()
    return x


def test_pvalues_uniform_under_the_null(ctx):
    """160 datasets of the law (alpha uniform on [1.8, 3.2], n in
    [200, 2000]), each tested with B = 500 bootstrap replicates (another
    seed, so independent draws).  The p-values, multiples of 1/500, must look
    uniform: Kolmogorov-Smirnov p > 1e-3, mean within 0.06 of 1/2 (its
    standard error is 0.023), and about a tenth below 0.1."""
    from scipy import stats
    rng = np.random.default_rng(21)
    ps = []
    for k in range(160):
        a = float(rng.uniform(1.8, 3.2))
        n = int(rng.integers(200, 2001))
        x = _draws(ctx, a, n, 7, k)
        ps.append(ctx.bootstrap_pvalue(x, 500, seed=1000 + k, stream_id=k)["p_value"])
    ps = np.array(ps)
    assert stats.kstest(ps, "uniform").pvalue > 1e-3, np.sort(ps)
    assert abs(ps.mean() - 0.5) < 0.06
    assert 4 <= np.sum(ps < 0.1) <= 32


def test_pvalues_small_against_another_law(ctx):
    """Data from round(lognormal(1, 1)) + 1 (not a power law): with n = 5,000
    the test rejects at the 1 % level in every case."""
    rng = np.random.default_rng(5)
    for k in range(6):
        x = (np.rint(rng.lognormal(1.0, 1.0, 5000)) + 1).astype(np.int64)
        r = ctx.bootstrap_pvalue(x, 500, seed=77 + k, stream_id=k)
        assert r["p_value"] < 0.01, (k, r)
