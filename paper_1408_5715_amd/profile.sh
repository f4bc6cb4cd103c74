#!/usr/bin/env bash
# rocprofv3 evidence for the kernels of the 2,097,152-cell workload (bench.py
# with its default 1000-step jobs and the random-order timing skipped, so
# every step launch runs on the renumbered mesh): a kernel trace with per-kernel statistics, then one
# counter pass each for FETCH_SIZE and WRITE_SIZE, with a plain 256 MiB copy
# in the same run as the calibration.  Output: gpurun_out/prof_* under the
# repository root.  Summarise with: python -m paper_1408_5715_amd.profile_summary
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
OUT="$ROOT/gpurun_out"
mkdir -p "$OUT"
export TMPDIR=/tmp
cd /tmp
echo "[profile] kernel trace" >&2
timeout -k 10 300 rocprofv3 --kernel-trace --stats -f csv -d "$OUT/prof_trace" -o trace -- \
    python3 "$ROOT/bench.py" --steps 3 --warmup 1 --no-cpu-baseline --skip-random \
    > "$OUT/prof_trace.log" 2>&1
echo "[profile] FETCH_SIZE" >&2
timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -f csv -d "$OUT/prof_fetch" -o fetch -- \
    python3 "$ROOT/bench.py" --steps 1 --warmup 0 --fv-steps 20 --no-cpu-baseline --skip-random \
    --probe-copy > "$OUT/prof_fetch.log" 2>&1
echo "[profile] WRITE_SIZE" >&2
timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -f csv -d "$OUT/prof_write" -o write -- \
    python3 "$ROOT/bench.py" --steps 1 --warmup 0 --fv-steps 20 --no-cpu-baseline --skip-random \
    --probe-copy > "$OUT/prof_write.log" 2>&1
echo "[profile] done" >&2
