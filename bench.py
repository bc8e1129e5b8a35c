"""Benchmark: Monte Carlo replicates per second (draw + MLE + KS + quantile
selection) for the n = 1000 slice of the full critical-value table (9
exponents 1.5..3.5 x n = 1000 x R = 100,000), batched (one persistent launch)
vs plain (one launch per cell), plus fit latency.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  A step is one call of zpl_simulate_cells on the whole
slice: table build, every replicate's draws, histogram, MLE and KS, and the
per-cell order statistics, with inputs (the cell list) resident; the host
reads back the quantiles each step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "MC replicates/sec (sample+MLE+KS) batched vs plain at n=1000; p99 fit latency"
QS = [(9, 10), (95, 100), (99, 100), (999, 1000)]

# Algorithmic VALU work model (ops per draw and per replicate):
# Philox4x32-10 = 10 rounds x (2 32x32->64 multiplies as 2 ops each + 2
# three-way xors as 2 ops each) = 80 ops per block of 2 draws; the 53-bit
# uniform 3 ops; guide lookup + table compare 4 ops; histogram update 2 ops.
OPS_PER_DRAW = 40 + 3 + 4 + 2
# MLE (about 5 Newton steps of 17 exp-equivalents x 20 ops) + KS + sums.
OPS_PER_REPLICATE = 2000
# Each 32x32->64 multiply of Philox is counted as two full-rate lane-ops (a low
# and a high product, one issue cycle per wave64 instruction on SIMD16 each).
INT_MUL_NOTE = "32x32->64 multiply = 2 full-rate lane-ops (low and high product)"
# VALU lane-op peak: 256 CUs x 64 lanes x 2.4 GHz.
PEAK_OPS = 256 * 64 * 2.4e9
# Heavy tails add, per replicate (expected counts under the law, see heavy_ops):
# a tail draw (x > 4096: a Philox block for the proposal and about five FP64
# transcendentals for the floored Pareto and its acceptance test);
# a distinct value above 16 (the KS terms: one Euler-Maclaurin survival value,
# one power, two terms); a value above the 1024-bin histogram (its FP64 log
# for S above the 4097-entry log table, and its share of a comparison sort).
OPS_TAIL_DRAW = 80 + 5 * 25
OPS_KS_VALUE = 60 + 25 + 5
OPS_OVERFLOW_LOG = 30
OPS_COMPARE = 4


def law_counts(alpha, n, kmax_sum=1 << 20):
    """Expected per-replicate counts of n draws from p(k) = k^-alpha/zeta(alpha):
    distinct values above 16, values above 1024 and above 4096 (the head summed
    directly, the far tail by n p(k) through the Hurwitz zeta)."""
    import numpy as np
    from scipy.special import zeta
    z = zeta(alpha, 1)
    k = np.arange(1, kmax_sum + 1, dtype=np.float64)
    p = k ** -alpha / z
    present = -np.expm1(n * np.log1p(-p))  # 1 - (1 - p)^n
    distinct16 = present[16:].sum() + n * zeta(alpha, kmax_sum + 1) / z
    above = lambda h: n * zeta(alpha, h + 1) / z  # noqa: E731
    return {"distinct_above_16": float(distinct16), "above_1024": float(above(1024)),
            "above_4096": float(above(4096))}


def heavy_ops(alpha, n):
    """Algorithmic lane-ops of one replicate in the heavy-tail regime: the
    headline model (draws and the fixed MLE/KS share) plus the expected tail
    draws, KS values above 16 and overflow values (log and sort comparisons)."""
    import math
    c = law_counts(alpha, n)
    m = c["above_1024"]
    return (n * OPS_PER_DRAW + OPS_PER_REPLICATE + c["above_4096"] * OPS_TAIL_DRAW
            + c["distinct_above_16"] * OPS_KS_VALUE
            + m * (OPS_OVERFLOW_LOG + OPS_COMPARE * max(math.log2(max(m, 2.0)), 1.0)))
# Autotuning grid: the table's exponents x sample sizes spanning 10..1e5.
TUNE_ALPHAS = [1.5 + 0.25 * i for i in range(9)]
TUNE_NS = [10, 30, 100, 300, 1000, 3000, 10000, 30000, 100000]


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


PROFILE = ROOT / "profiles" / "k_simulate_table_n1000.md"
HEAVY_PROFILE = ROOT / "profiles" / "k_heavy_heavy_tail.md"
# the device code's sources and the build script (its compiler flags)
KERNEL_SOURCES = ["paper_1305_6738_amd/csrc/zpl_kernels.hip", "paper_1305_6738_amd/csrc/zpl_kernels.hpp",
                  "paper_1305_6738_amd/csrc/zpl_math.hpp", "paper_1305_6738_amd/csrc/zpl_exp2_table.hpp",
                  "paper_1305_6738_amd/_build.py"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update((ROOT / f).read_bytes())
    return h.hexdigest()[:16]


def _profile_fields(path):
    """key: value lines of a committed profile summary, or {} when the kernel
    sources changed since it was taken."""
    if not path.exists():
        return {}
    vals = {}
    for line in path.read_text().splitlines():
        if ":" in line and line.split(":", 1)[0].replace("_", "").isalnum() and \
                not line.startswith("|"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return vals


def profiled_traffic(path=None):
    """HBM bytes per launch of the profiled kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy of
    known size), or None when the kernel sources changed since it was taken."""
    try:
        return float(_profile_fields(path or PROFILE)["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def profiled_counters(path=None):
    """Measured fractions of the committed profile (current sources only):
    VALU busy at the measured clock, executed VALU lane-instructions per
    second against the lane-op peak, FP64 FLOP rate against 78.6 TFLOP/s."""
    v = _profile_fields(path or PROFILE)
    out = {}
    for k in ("valu_busy", "valu_lane_inst_frac", "fp64_frac", "clock_ghz", "waves_per_simd"):
        try:
            out["measured_" + k] = float(v[k])
        except (KeyError, ValueError):
            pass
    return out


def percentile(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v), p)) if len(v) else None


def cpu_model():
    """The host CPU's model name (first "model name" line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cells, target_s=12.0, single_s=6.0):
    """The oracle on a bounded sample of the same cells, on every host core
    and on one thread: the first replicates of every cell, each run sized by
    a pilot to take about target_s (all cores) or single_s (one thread)
    seconds, at most the whole workload."""
    import oracle
    oracle.build(force=False)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    rmax = min(c[2] for c in cells)

    def timed(threads, budget_s, pilot):
        t0 = time.perf_counter()
        for (a, n, R, seed, st) in cells:
            oracle.simulate(a, n, seed, st, 0, pilot, nthreads=threads)
        tp = time.perf_counter() - t0
        reps = int(max(pilot, min(rmax, pilot * budget_s / max(tp, 1e-3))))
        t0 = time.perf_counter()
        for (a, n, R, seed, st) in cells:
            oracle.simulate(a, n, seed, st, 0, reps, nthreads=threads)
        return reps, time.perf_counter() - t0

    reps, dt = timed(cores, target_s, 256)
    reps1, dt1 = timed(1, single_s, 16)
    return {"value": len(cells) * reps / dt, "unit": "replicates/s", "cores": cores,
            "kind": "oracle",
            "sample": "first %d replicates of each of the %d cells (%.1f s on %d threads); "
                      "single thread: first %d of each (%.1f s)"
                      % (reps, len(cells), dt, cores, reps1, dt1),
            "single_thread_value": len(cells) * reps1 / dt1,
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def fit_latency(ctx, n_req=200):
    from inputs import serving_requests
    reqs = serving_requests(duration_s=1e9, qps=1.0, seed=11, max_requests=n_req)
    lat = []
    for (_, x, _, _) in reqs:
        t0 = time.perf_counter()
        ctx.fit(x)
        lat.append((time.perf_counter() - t0) * 1e3)
    return {"p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "requests": len(lat),
            "what": "zpl_fit of a host int64 dataset (n log-uniform 50..1e5), H2D included"}


def serving(ctx, qps=200.0, seconds=60.0, B=2500, budget=8 << 30, max_batch=0, seed=7):
    """Poisson request stream served with continuous batching (zpl_serve_*):
    each request fits its dataset and returns a B-replicate bootstrap p-value.
    Latency and queueing are measured by the library from submit to results
    ready (queue: submit to admission)."""
    from inputs import serving_requests
    reqs = serving_requests(duration_s=seconds, qps=qps, seed=seed)
    ctx.serve_start(mem_budget_bytes=budget, max_batch=max_batch)
    tickets = []
    t0 = time.perf_counter()
    try:
        for k, (ta, x, _, _) in enumerate(reqs):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            tickets.append(ctx.serve_submit(x, B, seed=k, stream_id=k))
        lat, qms, bs, launches, bad = [], [], [], [], 0
        for t in tickets:
            r = ctx.serve_poll(t, wait_ms=120000)
            if r is None or r["status"] != 0:
                bad += 1
                continue
            lat.append(r["latency_ms"])
            qms.append(r["queue_ms"])
            bs.append(r["batch_size"])
            launches.append(r["launches"])
        elapsed = time.perf_counter() - t0
    finally:
        ctx.serve_stop()
    return {"qps_offered": qps, "seconds": seconds, "requests": len(tickets), "failed": bad,
            "sustained_qps": len(tickets) / elapsed, "B": B,
            "budget_bytes": budget, "max_active": max_batch or 256,
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "queue_p50_ms": percentile(qms, 50), "queue_p99_ms": percentile(qms, 99),
            "queued_over_1ms": int(sum(1 for q in qms if q > 1.0)),
            "mean_batch": sum(bs) / max(len(bs), 1),
            "mean_launches": sum(launches) / max(len(launches), 1),
            "what": "Poisson %g/s, n log-uniform 50..1e5 (90%% Zipf, 10%% lognormal), "
                    "fit + B=%d bootstrap per request, continuous batching" % (qps, B)}


def config_runs(ctx, stream, torch):
    """One timed call (after one untimed) of each configuration beside the
    headline: the full table, the uneven batch, the heavy tails, and two
    slices of the truncated law's tables (n = 1000, 12 exponents)."""
    from inputs import table_cells, uneven_cells, heavy_tail
    gammas = [0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 3.5, 4.0]
    runs = {
        "full_table": ("9 alphas x n in {10..10000}, R = 100,000", table_cells(R=100000)),
        "uneven_batch": ("4,096 cells, n log-uniform [10, 1e5], alpha U(1.5, 3.5), R = 10,000",
                         uneven_cells(count=4096, R=10000)),
        "heavy_tail": ("alpha in {1.2, 1.3, 1.4, 1.5}, n = 10,000, R = 100,000", heavy_tail(R=100000)),
        "truncated_K20": ("truncated law K = 20: 12 exponents 0.25..4, n = 1000, R = 100,000",
                          [(g, 1000, 100000, 42, i, 20) for i, g in enumerate(gammas)]),
        "truncated_K1000": ("truncated law K = 1000: 12 exponents 0.25..4, n = 1000, R = 100,000",
                            [(g, 1000, 100000, 42, i, 1000) for i, g in enumerate(gammas)]),
    }
    out = {}
    for name, (what, cells) in runs.items():
        R = sum(c[2] for c in cells)
        ctx.simulate_cells(cells, quantiles=QS, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.simulate_cells(cells, quantiles=QS, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        tm = ctx.timing()
        draws = sum(c[1] * c[2] for c in cells)
        out[name] = {"what": what, "cells": len(cells), "replicates": R, "ms": ms,
                     "replicates_per_s": R / (ms / 1e3), "draws_per_s": draws / (ms / 1e3),
                     "kernel_ms": tm}
        if name == "heavy_tail":
            out[name]["roofline"] = heavy_roofline(cells, tm)
        progress("%s: %.1f ms" % (name, ms))
    return out


def heavy_roofline(cells, tm):
    """Roofline of the heavy-tail configuration: the heavy_ops model over
    every replicate against the simulation launches' time (HIP events: the
    lane/wave launch plus the heavy launch, which runs most of these cells),
    and the counters of the committed k_heavy profile while it is current."""
    ops = sum(R * heavy_ops(a, n) for (a, n, R, s, st) in cells)
    sec = (tm["simulate"] + tm["heavy"]) / 1e3
    r = {"bound": "alu", "achieved": ops / sec / 1e12, "peak": PEAK_OPS / 1e12,
         "unit": "Tops/s", "frac": ops / sec / PEAK_OPS, "kernel": "k_heavy",
         "kernel_ms": tm["heavy"], "simulate_ms": tm["simulate"], "ops_per_launch": ops,
         "traffic": profiled_traffic(HEAVY_PROFILE),
         "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)"}
    r.update(profiled_counters(HEAVY_PROFILE))
    return r


PAPER_NS = [10, 20, 30, 40, 50, 100, 500, 1000, 2000, 3000, 4000, 5000, 10000, 20000, 50000]


def paper_tables(ctx, torch):
    """Every table of the paper at its own size: Table 1 (pure law, 8
    exponents) and Tables 2-6 (K = 20, 50, 100, 500, 1000; 12 exponents),
    15 sample sizes each, 10 runs of 50,000 replicates per entry, quantiles
    .90/.95/.99/.999 averaged over the runs (one zpl_critical_table call per
    table, timed end to end on the host)."""
    g1 = [1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 3.5, 4.0]
    gt = [0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 3.5, 4.0]
    qs = ((9, 10), (95, 100), (99, 100), (999, 1000))
    ctx.critical_table([2.0], [10], kmax=0, seeds=1, replicates=1000, quantiles=qs)
    torch.cuda.synchronize()
    out = {"tables": {}}
    total_s, total_r, total_d = 0.0, 0, 0
    for name, K, gs in [("table1", 0, g1), ("table2_K20", 20, gt), ("table3_K50", 50, gt),
                        ("table4_K100", 100, gt), ("table5_K500", 500, gt),
                        ("table6_K1000", 1000, gt)]:
        t0 = time.perf_counter()
        ctx.critical_table(gs, PAPER_NS, kmax=K, seeds=10, seed0=1, replicates=50000,
                           quantiles=qs)
        dt = time.perf_counter() - t0
        reps = len(gs) * len(PAPER_NS) * 10 * 50000
        draws = len(gs) * sum(PAPER_NS) * 10 * 50000
        out["tables"][name] = {"s": dt, "replicates_per_s": reps / dt}
        total_s += dt
        total_r += reps
        total_d += draws
        progress("%s: %.2f s" % (name, dt))
    out.update({"what": "Tables 1-6 at the paper's size: 1,020 entries x 10 runs x 50,000 "
                        "replicates, quantiles .90/.95/.99/.999",
                "seconds": total_s, "replicates": total_r, "draws": total_d,
                "replicates_per_s": total_r / total_s,
                "paper_context": "the paper reports just over 373 hours for these runs on "
                                 "two GeForce GTX 590 (context only: other hardware, other "
                                 "sampler and KS scan)"})
    return out


def cutoff_runs(ctx, torch):
    """The law with a lower cutoff xmin: one timed batched call over six
    cells (alpha in {2, 2.5, 3} x xmin in {10, 100}, n = 1000, R = 100,000;
    heavy form), and one timed KS-minimising scan of 1,000 candidate cutoffs
    over a device dataset of 100,000 values (30,000 uniform on 1..59 below
    70,000 draws of the law with cutoff 60 and alpha = 2.5, drawn by the
    library's own sampler)."""
    import numpy as np
    out = {}
    cells = [(a, 1000, 100000, 42, i, 0, xm)
             for i, (a, xm) in enumerate([(a, xm) for a in (2.0, 2.5, 3.0) for xm in (10, 100)])]
    R = sum(c[2] for c in cells)
    ctx.simulate_cells(cells[:1], quantiles=QS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.simulate_cells(cells, quantiles=QS)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out["cells"] = {"what": "alpha in {2, 2.5, 3} x xmin in {10, 100}, n = 1000, R = 100,000",
                    "replicates": R, "ms": ms, "replicates_per_s": R / (ms / 1e3)}
    progress("cutoff cells: %.1f ms" % ms)
    rng = np.random.default_rng(7)
    body = torch.from_numpy(rng.integers(1, 60, size=30000).astype(np.int64)).cuda()
    tail = torch.zeros(70000, dtype=torch.int64, device="cuda")
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx.sample_draws(2.5, 70000, 7, 0, 0, 1, tail, fl, xmin=60)
    x = torch.cat([body, tail])
    cand = np.arange(1, 1001, dtype=np.int64)
    ctx.fit_scan(x, cand[:8])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.fit_scan(x, cand)
    ms = (time.perf_counter() - t0) * 1e3
    out["scan"] = {"what": "1,000 candidate cutoffs over 100,000 values (device input)",
                   "ms": ms, "candidates_per_s": cand.size / (ms / 1e3),
                   "chosen_xmin": int(cand[r["best"]]),
                   "alpha_hat": float(r["alpha_hat"][r["best"]])}
    progress("xmin scan: %.1f ms, chose %d" % (ms, cand[r["best"]]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replicates", type=int, default=100000)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the batched timed region (for profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-tables", action="store_true",
                    help="skip the timed run of all six tables at the paper's size")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--tune", default="measure",
                    help="'measure' (autotune before timing), 'none' (built-in rule) or "
                         "the path of a saved tuning table")
    ap.add_argument("--tune-out", default=None, help="save the measured tuning table here")
    ap.add_argument("--workload", default="table_n1000", choices=["table_n1000", "heavy_tail"],
                    help="cells of the timed region: the headline n = 1000 table slice, or "
                         "the heavy tails (alpha 1.2..1.5, n = 10,000; for profiling k_heavy)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device once (a kernel of known "
                         "traffic that scales the profiler's FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    from inputs import table_slice
    from paper_1305_6738_amd import Context, cell_array, load_tuning, plan_forms, save_tuning

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        progress("copy probe: %d MiB" % args.copy_probe_mib)
    if args.workload == "heavy_tail":
        from inputs import heavy_tail
        cells = heavy_tail(R=args.replicates)
    else:
        cells = table_slice(n=1000, R=args.replicates)
    total_R = sum(c[2] for c in cells)
    ctx = Context(0)
    d = torch.empty(total_R, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    tuning = {"source": args.tune}
    if args.tune == "measure":
        t0 = time.perf_counter()
        table = ctx.autotune(TUNE_ALPHAS, TUNE_NS, stream=stream)
        tuning.update(seconds=time.perf_counter() - t0,
                      grid="%d alphas x %d n" % (len(TUNE_ALPHAS), len(TUNE_NS)))
        progress("autotune: %.2f s" % tuning["seconds"])
        if args.tune_out:
            save_tuning(args.tune_out, table)
    elif args.tune != "none":
        table = load_tuning(args.tune)
        ctx.set_tuning(table)
    else:
        table = None
    tuning["forms"] = plan_forms(cells, table)
    ctx.set_timing(True)
    cs = cell_array(cells)  # converted once; every call below passes this zpl_cell array

    for _ in range(args.warmup):
        ctx.simulate_cells(cs, quantiles=QS, d_out=d, stream=stream)
    torch.cuda.synchronize()
    progress("warmup done (%d steps)" % args.warmup)
    sim_ms, all_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q = ctx.simulate_cells(cs, quantiles=QS, d_out=d, stream=stream)
        tm = ctx.timing()
        sim_ms.append(tm["simulate"] + tm["heavy"])
        all_ms.append(tm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = total_R / (ms_per_step / 1e3)
    progress("timed region: %.3f ms/step, %.4g replicates/s" % (ms_per_step, value))

    # dominant kernel: the persistent simulation launch
    sim_avg_ms = sum(sim_ms) / len(sim_ms)
    if args.workload == "heavy_tail":
        roofline = heavy_roofline(cells, {k: sum(t[k] for t in all_ms) / len(all_ms)
                                          for k in all_ms[0]})
    else:
        ops = sum(R * (n * OPS_PER_DRAW + OPS_PER_REPLICATE) for (a, n, R, s, st) in cells)
        achieved = ops / (sim_avg_ms / 1e3)
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_OPS / 1e12,
                    "unit": "Tops/s", "frac": achieved / PEAK_OPS, "traffic": profiled_traffic(),
                    "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                    "kernel": "k_simulate", "kernel_ms": sim_avg_ms,
                    "ops_per_launch": ops, "int_multiply_rate": INT_MUL_NOTE}
        roofline.update(profiled_counters(PROFILE))

    out = {"metric": METRIC, "value": value, "unit": "replicates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": ("full-table slice n=1000: alpha 1.5..3.5 step 0.25 (9 cells) "
                                   "x R=%d, seed 42, batched persistent launch" % args.replicates)
                      if args.workload == "table_n1000" else
                      ("heavy tails: alpha 1.2, 1.3, 1.4, 1.5 x n=10000 x R=%d, seed 42, "
                       "batched persistent launch (profiling workload)" % args.replicates),
                      "n": cells[0][1], "cells": len(cells), "replicates_per_cell": args.replicates,
                      "quantiles": ["%d/%d" % qq for qq in QS], "launch": "batched"},
           "kernel_ms": {k: sum(t[k] for t in all_ms) / len(all_ms) for k in all_ms[0]},
           "tuning": tuning,
           "roofline": roofline}

    if not args.no_extras:
        # plain: one launch per cell
        nplain = max(3, args.steps // 4)
        ctx.simulate_cells(cs, quantiles=QS, d_out=d, launch="plain", stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nplain):
            ctx.simulate_cells(cs, quantiles=QS, d_out=d, launch="plain", stream=stream)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3 / nplain
        out["plain_value"] = total_R / (plain_ms / 1e3)
        out["plain_ms_per_step"] = plain_ms
        out["batched_over_plain"] = value / out["plain_value"]
        progress("plain: %.3f ms/step" % plain_ms)
        # batched launch replayed from a hipGraph
        ctx.simulate_cells(cs, quantiles=QS, d_out=d, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.simulate_cells(cs, quantiles=QS, d_out=d, use_graph=True, stream=stream)
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        out["graph_value"] = total_R / (g_ms / 1e3)
        progress("graph replay: %.3f ms/step" % g_ms)
        # the same batched launch under the built-in form rule (no table)
        if table is not None:
            ctx.set_tuning(None)
            ctx.simulate_cells(cs, quantiles=QS, d_out=d, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nplain):
                ctx.simulate_cells(cs, quantiles=QS, d_out=d, stream=stream)
            torch.cuda.synchronize()
            u_ms = (time.perf_counter() - t0) * 1e3 / nplain
            out["untuned_value"] = total_R / (u_ms / 1e3)
            out["untuned_forms"] = plan_forms(cells)
            ctx.set_tuning(table)
            progress("built-in form rule: %.3f ms/step" % u_ms)
        out["configs"] = config_runs(ctx, stream, torch)
        if not args.no_paper_tables:
            out["paper_tables"] = paper_tables(ctx, torch)
        out["cutoff"] = cutoff_runs(ctx, torch)
        out["fit_latency"] = fit_latency(ctx)
        progress("fit latency done")
        if args.serve_seconds > 0:
            out["serving"] = serving(ctx, seconds=args.serve_seconds)
            progress("serving: p50 %.2f ms p99 %.2f ms" % (out["serving"]["p50_ms"],
                                                          out["serving"]["p99_ms"]))
            # a load point where admission throttles: five times the rate,
            # 16 active slots and a 32 MiB budget (a request of 1e5 values
            # needs about 4.4 MB of fit memory, so only a few fit at once)
            out["serving_throttled"] = serving(ctx, qps=1000.0, seconds=8.0, budget=32 << 20,
                                               max_batch=16, seed=8)
            progress("serving (throttled): p50 %.2f ms p99 %.2f ms queue p99 %.2f ms" % (
                out["serving_throttled"]["p50_ms"], out["serving_throttled"]["p99_ms"],
                out["serving_throttled"]["queue_p99_ms"]))
        out["quantiles_first_cell"] = [float(v) for v in q[0]]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cells)
        progress("cpu baseline done")
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
