"""Cell lists and request streams for the five benchmark configurations.

The paper's only workload is its own simulation grid (Table 1: exponents x
sample sizes, 50,000 replicates each); these cells are synthetic stand-ins of
the same shape.  Streams are numbered so that each cell owns its Philox
stream: table cell (i_alpha, i_n) uses stream 10 * i_alpha + i_n."""
from __future__ import annotations

import numpy as np

TABLE_ALPHAS = [1.5 + 0.25 * i for i in range(9)]
TABLE_NS = [10, 20, 50, 100, 200, 500, 1000, 2000, 5000, 10000]
SEED = 42


def single_cell(R: int = 10000):
    """alpha = 2.5, n = 100, R = 10,000, seed 42."""
    return [(2.5, 100, R, SEED, 0)]


def table_cells(R: int = 100000, alphas=TABLE_ALPHAS, ns=TABLE_NS):
    """Full table: 9 exponents x 10 sample sizes."""
    return [(a, n, R, SEED, 10 * i + j) for i, a in enumerate(alphas) for j, n in enumerate(ns)]


def table_slice(n: int = 1000, R: int = 100000):
    """The cells of the full table at one sample size (n = 1000: 9 cells)."""
    j = TABLE_NS.index(n)
    return [(a, n, R, SEED, 10 * i + j) for i, a in enumerate(TABLE_ALPHAS)]


def uneven_cells(count: int = 4096, R: int = 10000, seed: int = SEED):
    """Uneven batch: n log-uniform on [10, 1e5], alpha uniform on [1.5, 3.5]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.rint(10.0 ** rng.uniform(1.0, 5.0, count)).astype(np.int64)
    a = rng.uniform(1.5, 3.5, count)
    return [(float(a[i]), int(n[i]), R, SEED, i) for i in range(count)]


def heavy_tail(R: int = 100000, n: int = 10000):
    """Heavy tails: alpha in {1.2, 1.3, 1.4, 1.5}, n = 10,000."""
    return [(a, n, R, SEED, 100 + i) for i, a in enumerate([1.2, 1.3, 1.4, 1.5])]


def serving_requests(duration_s: float = 60.0, qps: float = 200.0, seed: int = 7,
                     n_lo: int = 50, n_hi: int = 100000, zipf_frac: float = 0.9,
                     max_requests: int = 1 << 30):
    """Poisson arrivals; each request an int64 dataset with n log-uniform on
    [n_lo, n_hi]: with probability zipf_frac a Zipf(alpha) sample (numpy's
    generator, alpha uniform on [1.5, 3.5]), otherwise round(lognormal(1, 1)) + 1.
    Returns a list of (arrival_time_s, dataset, kind, alpha or None)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    while len(out) < max_requests:
        t += rng.exponential(1.0 / qps)
        if t >= duration_s:
            break
        n = int(np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        if rng.random() < zipf_frac:
            a = float(rng.uniform(1.5, 3.5))
            x = rng.zipf(a, size=n).astype(np.int64)
            out.append((t, x, "zipf", a))
        else:
            x = (np.rint(rng.lognormal(1.0, 1.0, size=n)) + 1).astype(np.int64)
            out.append((t, x, "lognormal", None))
    return out
