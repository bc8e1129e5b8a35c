"""Summarise the output of profile.sh (rocprofv3 CSV files) as Markdown: one
kernel's average duration, its HBM traffic per launch (FETCH_SIZE and
WRITE_SIZE scaled by a copy of known size), the clock measured over its
dispatches (GRBM_COUNT / duration), and VALU / FP64 / LDS / occupancy
fractions from the SQ counters at that clock.

    python profile_summary.py OUT_DIR KERNEL "WORKLOAD TITLE" "BENCH ARGS" > summary.md
"""
import collections
import csv
import hashlib
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent
COPY_MIB = 256
NOMINAL_HZ = 2.4e9
N_CU, SIMD_PER_CU = 256, 4
STEPS = 5  # the timed steps of profile.sh's bench command
# the device code's sources and the build script (its compiler flags)
SOURCES = ["paper_1305_6738_amd/csrc/zpl_kernels.hip", "paper_1305_6738_amd/csrc/zpl_kernels.hpp",
           "paper_1305_6738_amd/csrc/zpl_math.hpp", "paper_1305_6738_amd/csrc/zpl_exp2_table.hpp",
           "paper_1305_6738_amd/_build.py"]


def source_hash():
    h = hashlib.sha256()
    for f in SOURCES:
        h.update((ROOT / f).read_bytes())
    return h.hexdigest()[:16]


def counters(d):
    """{dispatch id: (kernel name, {counter: value})}"""
    out = collections.OrderedDict()
    for r in csv.DictReader(open(Path(d) / "run_counter_collection.csv")):
        k = int(r["Dispatch_Id"])
        name, c = out.get(k, (r["Kernel_Name"], {}))
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        out[k] = (name, c)
    return out


def num_xcc(d):
    """XCDs (accelerator complex dies) of the GPU agent: block counters such as
    GRBM_COUNT are summed over them."""
    for r in csv.DictReader(open(Path(d) / "run_agent_info.csv")):
        if r.get("Agent_Type") == "GPU":
            return max(int(r.get("Num_Xcc", 1) or 1), 1)
    return 1


def dispatch_seconds(d, key):
    """{dispatch id: duration in s} of the kernel's dispatches in a counter run
    (its own timestamps: counters serialise the dispatches)."""
    out = {}
    for r in csv.DictReader(open(Path(d) / "run_counter_collection.csv")):
        if key in r["Kernel_Name"]:
            out[int(r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    return out


def last_dispatches(cs, key, count):
    sel = [(k, c) for k, (n, c) in cs.items() if key in n]
    return [c for _, c in sel[-count:]]


def main(out_dir, kernel, title, bench_args):
    out = Path(out_dir)
    trace = list(csv.DictReader(open(out / "trace" / "run_kernel_trace.csv")))
    sim = [r for r in trace if kernel in r["Kernel_Name"]]
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9 for r in sim[-STEPS:]]
    dur = sum(durs) / len(durs)
    stats = list(csv.DictReader(open(out / "trace" / "run_kernel_stats.csv")))
    fetch, write = counters(out / "fetch"), counters(out / "write")
    copy_f = [c for _, (n, c) in fetch.items() if "copyBuffer" in n and c.get("FETCH_SIZE", 0) > 1e5]
    copy_w = [c for _, (n, c) in write.items() if "copyBuffer" in n and c.get("WRITE_SIZE", 0) > 1e5]
    kib = COPY_MIB * 1024.0
    sf = kib / copy_f[0]["FETCH_SIZE"] if copy_f else 1.0
    sw = kib / copy_w[0]["WRITE_SIZE"] if copy_w else 1.0
    f_k = [c["FETCH_SIZE"] for c in last_dispatches(fetch, kernel, STEPS)]
    w_k = [c["WRITE_SIZE"] for c in last_dispatches(write, kernel, STEPS)]
    fb = sum(f_k) / len(f_k) * sf * 1024.0
    wb = sum(w_k) / len(w_k) * sw * 1024.0
    sq = last_dispatches(counters(out / "sq"), kernel, STEPS)[-1]
    sq2 = last_dispatches(counters(out / "sq2"), kernel, STEPS)[-1]
    # the clock over the kernel's last counted dispatch: GRBM_COUNT ticks once
    # per GPU clock on each XCD and the counter reads the sum over the XCDs
    xcc = num_xcc(out / "sq2")
    d2 = dispatch_seconds(out / "sq2", kernel)
    d2s = d2[max(d2)] if d2 else dur
    clock = sq2["GRBM_COUNT"] / xcc / d2s if sq2.get("GRBM_COUNT") else NOMINAL_HZ
    gui = sq2.get("GRBM_GUI_ACTIVE", 0.0) / max(sq2.get("GRBM_COUNT", 0.0), 1.0)
    simd_cycles = dur * clock * N_CU * SIMD_PER_CU
    cu_cycles = dur * clock * N_CU
    valu_busy = sq["SQ_ACTIVE_INST_VALU"] * 4.0 / simd_cycles
    lane_util = sq["SQ_THREAD_CYCLES_VALU"] / (sq["SQ_ACTIVE_INST_VALU"] * 64.0)
    inst_frac = sq["SQ_INSTS_VALU"] * 64.0 / (dur * clock * N_CU * 64.0)
    fp64 = sq["SQ_INSTS_VALU_FLOPS_FP64"] / dur / 78.6e12
    lds_busy = sq["SQ_LDS_IDX_ACTIVE"] / cu_cycles
    conflict = sq["SQ_LDS_BANK_CONFLICT"] / max(sq["SQ_LDS_IDX_ACTIVE"], 1.0)
    waves_per_simd = sq["SQ_WAVE_CYCLES"] * 4.0 / simd_cycles
    p = print
    p("# %s on %s, MI355X" % (kernel, title))
    p()
    p("Made by `paper_1305_6738_amd/profile.sh` (rocprofv3 on `bench.py %s`), summarised by "
      "`paper_1305_6738_amd/profile_summary.py`." % bench_args)
    p()
    p("kernel_source_sha256: `%s`" % source_hash())
    p()
    p("| Figure | Value |")
    p("|---|---|")
    p("| %s average duration, timed steps (kernel trace) | %.3f ms |" % (kernel, dur * 1e3))
    for r in stats:
        if kernel in r["Name"]:
            p("| %s average over all dispatches (rocprofv3 --stats) | %.3f ms (%s calls) |"
              % (kernel, float(r["AverageNs"]) * 1e-6, r["Calls"]))
    p("| clock over the dispatch (GRBM_COUNT / %d XCDs / duration); GUI active share | %.3f GHz; %.1f %% |"
      % (xcc, clock / 1e9, 100 * gui))
    p("| copy probe: FETCH_SIZE / WRITE_SIZE read for %d MiB | %.0f / %.0f KiB (scale %.3f / %.3f) |"
      % (COPY_MIB, copy_f[0]["FETCH_SIZE"] if copy_f else 0, copy_w[0]["WRITE_SIZE"] if copy_w else 0, sf, sw))
    p("| HBM bytes fetched per launch (scaled) | %.4g |" % fb)
    p("| HBM bytes written per launch (scaled) | %.4g |" % wb)
    p("| VALU busy (active VALU cycles / SIMD cycles) | %.1f %% |" % (100 * valu_busy))
    p("| VALU lane utilisation (thread cycles / 64 per active cycle) | %.1f %% |" % (100 * lane_util))
    p("| executed VALU lane-instructions / lane-op peak at that clock | %.1f %% |" % (100 * inst_frac))
    p("| FP64 FLOP rate / 78.6 TFLOP/s | %.2f %% |" % (100 * fp64))
    p("| LDS busy (SQ_LDS_IDX_ACTIVE / CU cycles) | %.1f %% |" % (100 * lds_busy))
    p("| LDS bank-conflict cycles / LDS active cycles | %.1f %% |" % (100 * conflict))
    p("| waves resident per SIMD (occupancy) | %.2f |" % waves_per_simd)
    p("| VALU / SALU / LDS instructions per launch (wave-level) | %.4g / %.4g / %.4g |"
      % (sq["SQ_INSTS_VALU"], sq2["SQ_INSTS_SALU"], sq2["SQ_INSTS_LDS"]))
    p("| INT32 / INT64 VALU instructions | %.4g / %.4g |"
      % (sq2["SQ_INSTS_VALU_INT32"], sq2["SQ_INSTS_VALU_INT64"]))
    p("| SQ_WAIT_INST_ANY / SQ_BUSY_CYCLES | %.4g / %.4g |"
      % (sq2["SQ_WAIT_INST_ANY"], sq2["SQ_BUSY_CYCLES"]))
    p()
    p("traffic_bytes_per_launch: `%.6g`" % (fb + wb))
    p("clock_ghz: `%.4f`" % (clock / 1e9))
    p("valu_busy: `%.4f`" % valu_busy)
    p("valu_lane_inst_frac: `%.4f`" % inst_frac)
    p("fp64_frac: `%.5f`" % fp64)
    p("waves_per_simd: `%.3f`" % waves_per_simd)
    p()
    p("Cycle-based fractions use the measured clock; SQ counters from the last timed launch, "
      "traffic averaged over the timed launches.")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], sys.argv[3], sys.argv[4])
