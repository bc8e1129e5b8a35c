"""Reference (oracle) implementation -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU implementation (C, FP64) of the Monte Carlo KS critical-value
method of Rappos & Robert (2013) for the pure discrete power law and its
truncated variant on 1..K, used to check the GPU library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the product path never
does.  The C source is ``zpl_oracle.c``; this module builds it with gcc and
wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "zpl_oracle.c"
_LIB = _HERE / "libzpl_oracle.so"

TABLE_H = 4096
FLAG_ALL_ONES = 1
FLAG_TAIL_CAPPED = 2
FLAG_BISECT = 4
FLAG_NOCONV = 8

_lib = None


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (plain -O2, no vector intrinsics)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-Wno-unused-parameter", str(_SRC), "-o", str(tmp),
               "-lquadmath", "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def compile_variant(src: Path, out: Path) -> Path:
    """Compile another copy of the oracle source (used by tests that plant
    mistakes in the oracle to check that the pins catch them)."""
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-I", str(_HERE), str(src),
                    "-o", str(out), "-lquadmath", "-lm", "-lpthread"], check=True,
                   capture_output=True)
    return out


class use_library:
    """Context manager: route this module's functions to another build."""

    def __init__(self, path: Path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(C.CDLL(str(self.path)))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        _lib = _bind(C.CDLL(str(_LIB)))
    return _lib


def _bind(L):
    """Declare the C signatures on a loaded oracle library."""
    if True:  # keeps the declarations' indentation
        d, i64, u32, u64 = C.c_double, C.c_int64, C.c_uint32, C.c_uint64
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_u53.argtypes = [u32, u32]
        L.orc_u53.restype = d
        L.orc_hurwitz3.argtypes = [d, d, P(d)]
        L.orc_zeta3.argtypes = [d, P(d)]
        L.orc_cdf.argtypes = [d, i64]
        L.orc_cdf.restype = d
        L.orc_cdf_table.argtypes = [d, P(d), C.c_int]
        L.orc_draw.argtypes = [d, P(d), u64, u32, u32, u32, P(u32)]
        L.orc_draw.restype = i64
        L.orc_tail_draw.argtypes = [d, u64, u32, u32, u32, P(u32)]
        L.orc_tail_draw.restype = i64
        L.orc_sample.argtypes = [d, P(d), i64, u64, u32, u32, P(i64), P(u32)]
        L.orc_mle_last_iters.argtypes = []
        L.orc_mle_last_iters.restype = C.c_int
        L.orc_mle.argtypes = [d, P(u32)]
        L.orc_mle.restype = d
        L.orc_fit.argtypes = [P(i64), i64, P(d), P(d), P(d), P(u32)]
        L.orc_fit.restype = C.c_int
        L.orc_simulate.argtypes = [d, i64, u64, u32, i64, i64, P(d), P(d), P(d),
                                   P(u32), P(u64), P(i64), C.c_int]
        L.orc_simulate.restype = C.c_int
        L.orc_quantile.argtypes = [P(d), i64, u32, u32]
        L.orc_quantile.restype = d
        L.orc_bootstrap_pvalue.argtypes = [P(i64), i64, i64, u64, u32, P(d), P(d),
                                           P(d), P(u32), C.c_int]
        L.orc_bootstrap_pvalue.restype = C.c_int
        ci = C.c_int
        L.orc_tz_norm3.argtypes = [d, ci, P(d)]
        L.orc_tz_cdf_table.argtypes = [d, ci, P(d)]
        L.orc_tz_cdf_table.restype = ci
        L.orc_tz_draw.argtypes = [P(d), ci, u64, u32, u32, u32]
        L.orc_tz_draw.restype = i64
        L.orc_tz_mle.argtypes = [d, ci, P(u32)]
        L.orc_tz_mle.restype = d
        L.orc_tz_fit.argtypes = [P(i64), i64, ci, P(d), P(d), P(d), P(u32)]
        L.orc_tz_fit.restype = ci
        L.orc_tz_simulate.argtypes = [d, ci, i64, u64, u32, i64, i64, P(d), P(d), P(d),
                                      P(u32), P(u64), P(i64), ci]
        L.orc_tz_simulate.restype = ci
        L.orc_hz_cdf_table.argtypes = [d, i64, P(d)]
        L.orc_hz_draw.argtypes = [d, i64, P(d), u64, u32, u32, u32, P(u32)]
        L.orc_hz_draw.restype = i64
        L.orc_hz_mle.argtypes = [d, i64, P(u32)]
        L.orc_hz_mle.restype = d
        L.orc_hz_fit.argtypes = [P(i64), i64, i64, P(i64), P(d), P(d), P(d), P(u32)]
        L.orc_hz_fit.restype = ci
        L.orc_hz_scan.argtypes = [P(i64), i64, P(i64), ci, P(d), P(d), P(i64), P(u32)]
        L.orc_hz_scan.restype = ci
        L.orc_hz_simulate.argtypes = [d, i64, i64, u64, u32, i64, i64, P(d), P(d), P(d),
                                      P(u32), P(u64), P(i64), ci]
        L.orc_hz_simulate.restype = ci
    return L


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def u53(hi: int, lo: int) -> float:
    return lib().orc_u53(hi, lo)


def hurwitz3(s: float, q: float):
    out = np.zeros(3)
    lib().orc_hurwitz3(s, q, _ptr(out, C.c_double))
    return out


def zeta3(s: float):
    out = np.zeros(3)
    lib().orc_zeta3(s, _ptr(out, C.c_double))
    return out


def cdf(alpha: float, t: int) -> float:
    return lib().orc_cdf(alpha, int(t))


def cdf_table(alpha: float, H: int = TABLE_H) -> np.ndarray:
    T = np.zeros(H)
    lib().orc_cdf_table(alpha, _ptr(T, C.c_double), H)
    return T


def sample(alpha: float, n: int, seed: int, stream: int, rep: int):
    """n draws of one replicate in draw order -> (int64 array, flags)."""
    T = cdf_table(alpha)
    x = np.zeros(n, dtype=np.int64)
    f = C.c_uint32(0)
    lib().orc_sample(alpha, _ptr(T, C.c_double), n, seed, stream, rep,
                     _ptr(x, C.c_int64), C.byref(f))
    return x, f.value


def tail_draw(alpha: float, seed: int, stream: int, rep: int, i: int):
    f = C.c_uint32(0)
    x = lib().orc_tail_draw(alpha, seed, stream, rep, i, C.byref(f))
    return x, f.value


def mle_last_iters() -> int:
    """Iterations of the calling thread's last MLE solve (any of the laws)."""
    return int(lib().orc_mle_last_iters())


def mle(m: float):
    f = C.c_uint32(0)
    a = lib().orc_mle(m, C.byref(f))
    return a, f.value


def fit(x) -> dict:
    x = np.ascontiguousarray(x, dtype=np.int64)
    S, a, D = C.c_double(), C.c_double(), C.c_double()
    f = C.c_uint32(0)
    rc = lib().orc_fit(_ptr(x, C.c_int64), x.size, C.byref(S), C.byref(a), C.byref(D),
                       C.byref(f))
    if rc != 0:
        raise ValueError("oracle fit: invalid dataset (n < 1 or some x < 1)")
    return {"S": S.value, "alpha_hat": a.value, "D": D.value, "flags": f.value}


def simulate(alpha: float, n: int, seed: int, stream: int, rep_lo: int, count: int,
             nthreads: int = 0) -> dict:
    D = np.zeros(count)
    A = np.zeros(count)
    S = np.zeros(count)
    F = np.zeros(count, dtype=np.uint32)
    FP = np.zeros(count, dtype=np.uint64)
    XM = np.zeros(count, dtype=np.int64)
    rc = lib().orc_simulate(alpha, n, seed, stream, rep_lo, count,
                            _ptr(D, C.c_double), _ptr(A, C.c_double), _ptr(S, C.c_double),
                            _ptr(F, C.c_uint32), _ptr(FP, C.c_uint64), _ptr(XM, C.c_int64),
                            nthreads)
    if rc != 0:
        raise ValueError("oracle simulate: invalid cell")
    return {"D": D, "alpha_hat": A, "S": S, "flags": F, "fp": FP, "xmax": XM}


def quantile(D, num: int, den: int) -> float:
    D = np.ascontiguousarray(D, dtype=np.float64)
    return lib().orc_quantile(_ptr(D, C.c_double), D.size, num, den)


def bootstrap_pvalue(x, B: int, seed: int, stream: int, nthreads: int = 0) -> dict:
    x = np.ascontiguousarray(x, dtype=np.int64)
    a, D, p = C.c_double(), C.c_double(), C.c_double()
    f = C.c_uint32(0)
    rc = lib().orc_bootstrap_pvalue(_ptr(x, C.c_int64), x.size, B, seed, stream,
                                    C.byref(a), C.byref(D), C.byref(p), C.byref(f),
                                    nthreads)
    if rc != 0:
        raise ValueError("oracle bootstrap: invalid input")
    return {"alpha_hat": a.value, "D": D.value, "p_value": p.value, "flags": f.value}


# ---- truncated law on 1..K (Sect. 1 with a finite upper limit) -------------

def tz_norm3(g: float, K: int):
    out = np.zeros(3)
    lib().orc_tz_norm3(g, K, _ptr(out, C.c_double))
    return out


def tz_cdf_table(g: float, K: int) -> np.ndarray:
    T = np.zeros(K)
    if lib().orc_tz_cdf_table(g, K, _ptr(T, C.c_double)) != 0:
        raise ValueError("K must be >= 2")
    return T


def tz_sample(g: float, K: int, n: int, seed: int, stream: int, rep: int) -> np.ndarray:
    T = tz_cdf_table(g, K)
    return np.array([lib().orc_tz_draw(_ptr(T, C.c_double), K, seed, stream, rep, i)
                     for i in range(n)], dtype=np.int64)


def tz_mle(m: float, K: int):
    f = C.c_uint32(0)
    g = lib().orc_tz_mle(m, K, C.byref(f))
    return g, f.value


def tz_fit(x, K: int) -> dict:
    x = np.ascontiguousarray(x, dtype=np.int64)
    S, g, D = C.c_double(), C.c_double(), C.c_double()
    f = C.c_uint32(0)
    rc = lib().orc_tz_fit(_ptr(x, C.c_int64), x.size, K, C.byref(S), C.byref(g), C.byref(D),
                          C.byref(f))
    if rc != 0:
        raise ValueError("oracle tz_fit: invalid dataset (n < 1, K < 2 or x outside 1..K)")
    return {"S": S.value, "alpha_hat": g.value, "D": D.value, "flags": f.value}


def tz_simulate(g: float, K: int, n: int, seed: int, stream: int, rep_lo: int, count: int,
                nthreads: int = 0) -> dict:
    D = np.zeros(count)
    A = np.zeros(count)
    S = np.zeros(count)
    F = np.zeros(count, dtype=np.uint32)
    FP = np.zeros(count, dtype=np.uint64)
    XM = np.zeros(count, dtype=np.int64)
    rc = lib().orc_tz_simulate(g, K, n, seed, stream, rep_lo, count,
                               _ptr(D, C.c_double), _ptr(A, C.c_double), _ptr(S, C.c_double),
                               _ptr(F, C.c_uint32), _ptr(FP, C.c_uint64), _ptr(XM, C.c_int64),
                               nthreads)
    if rc != 0:
        raise ValueError("oracle tz_simulate: invalid cell")
    return {"D": D, "alpha_hat": A, "S": S, "flags": F, "fp": FP, "xmax": XM}


# ---- the law with a lower cutoff xmin (p(k) proportional to k^-alpha, k >= xmin) ----

def hz_cdf_table(alpha: float, xmin: int) -> np.ndarray:
    T = np.zeros(TABLE_H)
    lib().orc_hz_cdf_table(alpha, xmin, _ptr(T, C.c_double))
    return T


def hz_sample(alpha: float, xmin: int, n: int, seed: int, stream: int, rep: int):
    """n draws of one replicate in draw order -> (int64 array, flags)."""
    T = hz_cdf_table(alpha, xmin)
    f = C.c_uint32(0)
    x = np.array([lib().orc_hz_draw(alpha, xmin, _ptr(T, C.c_double), seed, stream, rep, i,
                                    C.byref(f)) for i in range(n)], dtype=np.int64)
    return x, f.value


def hz_mle(m: float, xmin: int):
    f = C.c_uint32(0)
    a = lib().orc_hz_mle(m, xmin, C.byref(f))
    return a, f.value


def hz_fit(x, xmin: int) -> dict:
    """Fit the values >= xmin: S, alpha_hat, D, flags and their count."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    S, a, D = C.c_double(), C.c_double(), C.c_double()
    m = C.c_int64(0)
    f = C.c_uint32(0)
    rc = lib().orc_hz_fit(_ptr(x, C.c_int64), x.size, xmin, C.byref(m), C.byref(S), C.byref(a),
                          C.byref(D), C.byref(f))
    if rc == -1:
        raise ValueError("oracle hz_fit: invalid dataset (n < 1, xmin < 1 or some x < 1)")
    if rc == -2:
        raise ValueError("oracle hz_fit: no value >= xmin")
    return {"S": S.value, "alpha_hat": a.value, "D": D.value, "flags": f.value, "n_tail": m.value}


def hz_scan(x, xmins) -> dict:
    """The KS-minimising xmin among the candidates: per-candidate fits and
    the index of the smallest D (the first on ties)."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    c = np.ascontiguousarray(xmins, dtype=np.int64)
    A = np.zeros(c.size)
    D = np.zeros(c.size)
    M = np.zeros(c.size, dtype=np.int64)
    F = np.zeros(c.size, dtype=np.uint32)
    best = lib().orc_hz_scan(_ptr(x, C.c_int64), x.size, _ptr(c, C.c_int64), c.size,
                             _ptr(A, C.c_double), _ptr(D, C.c_double), _ptr(M, C.c_int64),
                             _ptr(F, C.c_uint32))
    if best == -1:
        raise ValueError("oracle hz_scan: invalid input")
    return {"best": best, "alpha_hat": A, "D": D, "n_tail": M, "flags": F}


def hz_simulate(alpha: float, xmin: int, n: int, seed: int, stream: int, rep_lo: int,
                count: int, nthreads: int = 0) -> dict:
    D = np.zeros(count)
    A = np.zeros(count)
    S = np.zeros(count)
    F = np.zeros(count, dtype=np.uint32)
    FP = np.zeros(count, dtype=np.uint64)
    XM = np.zeros(count, dtype=np.int64)
    rc = lib().orc_hz_simulate(alpha, xmin, n, seed, stream, rep_lo, count,
                               _ptr(D, C.c_double), _ptr(A, C.c_double), _ptr(S, C.c_double),
                               _ptr(F, C.c_uint32), _ptr(FP, C.c_uint64), _ptr(XM, C.c_int64),
                               nthreads)
    if rc != 0:
        raise ValueError("oracle hz_simulate: invalid cell")
    return {"D": D, "alpha_hat": A, "S": S, "flags": F, "fp": FP, "xmax": XM}


# ---- a whole table (Sect. 3: how Tables 1-6 are built) ---------------------

def critical_table(gammas, ns, K: int = 0, seeds: int = 10, seed0: int = 1, R: int = 50000,
                   quantiles=((9, 10), (95, 100), (99, 100), (999, 1000)),
                   nthreads: int = 0):
    """Sect. 3's construction of a table: at every (N, gamma) entry, `seeds`
    independent runs of R replicates (run s: seed seed0 + s, stream
    i_n * len(gammas) + i_g), the quantile order statistic of each run's D
    values, and their mean over the runs (summed in run order, then divided
    by the number of runs).  K = 0 is the pure law (Table 1), else the law
    truncated to 1..K (Tables 2-6).  Returns (table [len(ns), len(gammas),
    n_q], per_run [len(ns), len(gammas), seeds, n_q])."""
    q = list(quantiles)
    runs = np.zeros((len(ns), len(gammas), seeds, len(q)))
    for i_n, n in enumerate(ns):
        for i_g, g in enumerate(gammas):
            stream = i_n * len(gammas) + i_g
            for s in range(seeds):
                if K:
                    D = tz_simulate(g, K, n, seed0 + s, stream, 0, R, nthreads)["D"]
                else:
                    D = simulate(g, n, seed0 + s, stream, 0, R, nthreads)["D"]
                runs[i_n, i_g, s] = [quantile(D, a, b) for a, b in q]
    table = np.zeros((len(ns), len(gammas), len(q)))
    for i_n in range(len(ns)):
        for i_g in range(len(gammas)):
            for k in range(len(q)):
                acc = 0.0
                for s in range(seeds):
                    acc += runs[i_n, i_g, s, k]
                table[i_n, i_g, k] = acc / seeds
    return table, runs
