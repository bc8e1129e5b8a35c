#!/bin/bash
# Profiles one of the benchmark's timed workloads on one GPU with rocprofv3:
#   1. kernel trace + per-kernel statistics (durations);
#   2. FETCH_SIZE and 3. WRITE_SIZE per dispatch (HBM traffic), each in a run
#      of its own, with a 256 MiB device-to-device copy first whose counters
#      scale the readings to bytes;
#   4./5. SQ counters and the clock (GRBM_COUNT) in two more runs.
# The shipped tuning table is loaded so that no autotuning probe launches mix
# into the statistics.
#   profile.sh [OUT_DIR] [table_n1000|heavy_tail]
# table_n1000 (default) profiles k_simulate on the headline slice, heavy_tail
# profiles k_heavy on the heavy-tail cells.  Output: OUT_DIR (default
# profile_out/ at the root), summary in OUT_DIR/summary.md.
set -o pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
OUT="${1:-$ROOT/profile_out}"
WL="${2:-table_n1000}"
mkdir -p "$OUT"
cd /tmp && export TMPDIR=/tmp
case "$WL" in
  table_n1000) KERNEL=k_simulate; TITLE="the n = 1000 table slice (9 cells x 100,000 replicates)";;
  heavy_tail) KERNEL=k_heavy; TITLE="the heavy tails (alpha 1.2, 1.3, 1.4, 1.5 x n = 10,000 x 100,000 replicates)";;
  *) echo "unknown workload $WL"; exit 2;;
esac
ARGS="--workload $WL --steps 5 --warmup 2 --no-extras --no-cpu-baseline --tune paper_1305_6738_amd/tuning/mi355x.json --copy-probe-mib 256"
RUNARGS="${ARGS/paper_1305_6738_amd\/tuning/$ROOT/paper_1305_6738_amd/tuning}"
echo "== kernel trace ($WL)"
timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "$OUT/trace" -o run -- \
  python3 "$ROOT/bench.py" $RUNARGS > "$OUT/trace.log" 2>&1 || exit $?
tail -1 "$OUT/trace.log" | cut -c1-200
SQ="SQ_WAVES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_INSTS_VALU_FLOPS_FP64 SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT"
SQ2="SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAIT_INST_ANY SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_BUSY_CYCLES GRBM_COUNT GRBM_GUI_ACTIVE"
for pass in "fetch:FETCH_SIZE" "write:WRITE_SIZE" "sq:$SQ" "sq2:$SQ2"; do
  name="${pass%%:*}"; ctrs="${pass#*:}"
  echo "== pmc $name"
  timeout -s KILL 180 rocprofv3 --pmc $ctrs --output-format csv -d "$OUT/$name" -o run -- \
    python3 "$ROOT/bench.py" $RUNARGS > "$OUT/$name.log" 2>&1 || exit $?
  tail -1 "$OUT/$name.log" | cut -c1-200
done
echo "== summary"
python3 "$ROOT/paper_1305_6738_amd/profile_summary.py" "$OUT" "$KERNEL" "$TITLE" "$ARGS" > "$OUT/summary.md" || exit $?
cat "$OUT/summary.md"
