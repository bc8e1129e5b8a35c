#!/bin/bash
# Profiles the benchmark's timed workload on one GPU with rocprofv3:
#   1. kernel trace + per-kernel statistics (durations);
#   2. FETCH_SIZE and 3. WRITE_SIZE per dispatch (HBM traffic), each in a run
#      of its own, with a 256 MiB device-to-device copy first whose counters
#      scale the readings to bytes.
# The shipped tuning table is loaded so that no autotuning probe launches mix
# into the statistics.  Output goes to $1 (default profile_out/ at the root).
set -o pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
OUT="${1:-$ROOT/profile_out}"
mkdir -p "$OUT"
cd /tmp && export TMPDIR=/tmp
ARGS="--steps 5 --warmup 2 --no-extras --no-cpu-baseline --tune $ROOT/paper_1305_6738_amd/tuning/mi355x.json --copy-probe-mib 256"
echo "== kernel trace"
timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/trace" -o run -- \
  python3 "$ROOT/bench.py" $ARGS > "$OUT/trace.log" 2>&1 || exit $?
tail -1 "$OUT/trace.log"
SQ="SQ_WAVES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_INSTS_VALU_FLOPS_FP64 SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT"
SQ2="SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAIT_INST_ANY SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_BUSY_CYCLES"
for pass in "fetch:FETCH_SIZE" "write:WRITE_SIZE" "sq:$SQ" "sq2:$SQ2"; do
  name="${pass%%:*}"; ctrs="${pass#*:}"
  echo "== pmc $name"
  timeout -s KILL 120 rocprofv3 --pmc $ctrs --output-format csv -d "$OUT/$name" -o run -- \
    python3 "$ROOT/bench.py" $ARGS > "$OUT/$name.log" 2>&1 || exit $?
  tail -1 "$OUT/$name.log"
done
echo "== summary"
python3 "$ROOT/paper_1305_6738_amd/profile_summary.py" "$OUT" > "$OUT/summary.md" || exit $?
head -5 "$OUT/summary.md"
