#!/usr/bin/env bash
# rocprofv3 evidence for the kernels of the 2,097,152-cell workload (bench.py
# with its default 1000-step jobs and the random-order timing skipped, so
# every step launch runs on the renumbered mesh): a kernel trace with per-kernel statistics, then one
# counter pass each for FETCH_SIZE and WRITE_SIZE, with a plain 256 MiB copy
# in the same run as the calibration, then L2 hits and misses of the step on
# the random order and on the renumbered order.  Output: prof_* under
# $FV_PROFILE_DIR (default: profile_out/ at the repository root).  Summarise
# with: python profile_summary.py (same FV_PROFILE_DIR)
#
# `profile.sh learned`: the same three runs for the learned-correction
# kernels (profile_learned.py: 20 corrected steps on the
# 1024 x 1024 mesh, 4 corrected adjoint steps on the 32-flow training batch),
# with MFMA counters in place of the byte counters.  Output lprof_*.
#
# `profile.sh renumber`: two counter passes (wave and instruction counters;
# texture-addresser, L1-to-L2 and clock counters) over one bench.py job of
# the 2,097,152-cell workload, for the renumbering kernels and the step.
# Output rprof_*.  Summarise with python profile_summary.py renumber.
#
# `profile.sh hbm [32|40]`: the step alone on the 2048 x 2048-quad mesh
# (8,388,608 cells, working set beyond the Infinity Cache; bench.py
# --workload hbm, coordinates on a 2^-32 grid, or 2^-40 for float64
# normals): a kernel trace, then FETCH_SIZE and WRITE_SIZE with the
# calibration copy.  Output hprof_*.  Summarise with python
# profile_summary.py hbm.
#
# `profile.sh orders`: the random / AM1 / Cuthill-McKee comparison on the
# 512 x 512-quad irregular mesh (tests/test_gpu_irregular.py) under the L2
# hit and miss counters.  Output oprof_*.  Summarise with
# python profile_summary.py orders.
set -euo pipefail
ROOT="$(cd "$(dirname "$0")" && pwd)"
OUT="${FV_PROFILE_DIR:-$ROOT/profile_out}"
mkdir -p "$OUT"
export TMPDIR=/tmp
export PYTHONPATH="$ROOT${PYTHONPATH:+:$PYTHONPATH}"
cd /tmp
if [ "${1:-}" = "renumber" ]; then
    # one job of bench.py (renumbering + 20 steps) under two counter passes
    JOB=(python3 "$ROOT/bench.py" --steps 1 --warmup 0 --fv-steps 20 --no-cpu-baseline --skip-random --hbm-N 0 --skip-batch)
    echo "[profile] renumber: SQ counters" >&2
    timeout -s KILL 120 rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY \
        SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_INSTS_VALU SQ_INSTS_VMEM_RD -f csv \
        -d "$OUT/rprof_sq" -o sq -- "${JOB[@]}" > "$OUT/rprof_sq.log" 2>&1
    echo "[profile] renumber: memory-path counters" >&2
    timeout -s KILL 120 rocprofv3 --pmc TA_TA_BUSY TA_ADDR_STALLED_BY_TC_CYCLES TCP_TCC_READ_REQ \
        TCP_TCC_READ_REQ_LATENCY GRBM_GUI_ACTIVE SQ_INSTS_LDS -f csv \
        -d "$OUT/rprof_mem" -o mem -- "${JOB[@]}" > "$OUT/rprof_mem.log" 2>&1
    echo "[profile] done" >&2
    exit 0
fi
if [ "${1:-}" = "hbm" ]; then
    # optional second argument: the coordinate grid (32: compact normals,
    # 40: float64 normals)
    HBM=(python3 "$ROOT/bench.py" --workload hbm --hbm-N 2048 --snap-bits "${2:-32}")
    echo "[profile] hbm: kernel trace" >&2
    timeout -k 10 300 rocprofv3 --kernel-trace --stats -f csv -d "$OUT/hprof_trace" -o trace -- \
        "${HBM[@]}" --fv-steps 200 > "$OUT/hprof_trace.log" 2>&1
    echo "[profile] hbm: FETCH_SIZE" >&2
    timeout -s KILL 180 rocprofv3 --pmc FETCH_SIZE -f csv -d "$OUT/hprof_fetch" -o fetch -- \
        "${HBM[@]}" --fv-steps 20 --probe-copy > "$OUT/hprof_fetch.log" 2>&1
    echo "[profile] hbm: WRITE_SIZE" >&2
    timeout -s KILL 180 rocprofv3 --pmc WRITE_SIZE -f csv -d "$OUT/hprof_write" -o write -- \
        "${HBM[@]}" --fv-steps 20 --probe-copy > "$OUT/hprof_write.log" 2>&1
    echo "[profile] done" >&2
    exit 0
fi
if [ "${1:-}" = "orders" ]; then
    # the order comparison on the 512 x 512 irregular mesh (a test: AM1 comes
    # from the CPU reference) under the L2 hit and miss counters
    echo "[profile] orders: L2 hits and misses per order" >&2
    timeout -s KILL 600 rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum -f csv -d "$OUT/oprof_l2" -o l2 -- \
        python3 -m pytest -q -s -m gpu -k orders "$ROOT/tests/test_gpu_irregular.py" > "$OUT/oprof_l2.log" 2>&1
    echo "[profile] done" >&2
    exit 0
fi
if [ "${1:-}" = "learned" ]; then
    echo "[profile] learned: kernel trace" >&2
    timeout -k 10 300 rocprofv3 --kernel-trace --stats -f csv -d "$OUT/lprof_trace" -o trace -- \
        python3 "$ROOT/profile_learned.py" --adjoint > "$OUT/lprof_trace.log" 2>&1
    echo "[profile] learned: MFMA counters" >&2
    timeout -s KILL 120 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_VALU_MFMA_MOPS_BF16 \
        SQ_VALU_MFMA_BUSY_CYCLES SQ_WAVES SQ_INSTS_LDS GRBM_GUI_ACTIVE -f csv -d "$OUT/lprof_mfma" \
        -o mfma -- python3 "$ROOT/profile_learned.py" --adjoint > "$OUT/lprof_mfma.log" 2>&1
    echo "[profile] learned: byte counters" >&2
    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -f csv -d "$OUT/lprof_fetch" -o fetch -- \
        python3 "$ROOT/profile_learned.py" --probe-copy > "$OUT/lprof_fetch.log" 2>&1
    echo "[profile] done" >&2
    exit 0
fi
echo "[profile] kernel trace" >&2
timeout -k 10 300 rocprofv3 --kernel-trace --stats -f csv -d "$OUT/prof_trace" -o trace -- \
    python3 "$ROOT/bench.py" --steps 3 --warmup 1 --no-cpu-baseline --skip-random --hbm-N 0 --skip-batch \
    > "$OUT/prof_trace.log" 2>&1
echo "[profile] FETCH_SIZE" >&2
timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -f csv -d "$OUT/prof_fetch" -o fetch -- \
    python3 "$ROOT/bench.py" --steps 1 --warmup 0 --fv-steps 20 --no-cpu-baseline --skip-random --hbm-N 0 --skip-batch \
    --probe-copy > "$OUT/prof_fetch.log" 2>&1
echo "[profile] WRITE_SIZE" >&2
timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -f csv -d "$OUT/prof_write" -o write -- \
    python3 "$ROOT/bench.py" --steps 1 --warmup 0 --fv-steps 20 --no-cpu-baseline --skip-random --hbm-N 0 --skip-batch \
    --probe-copy > "$OUT/prof_write.log" 2>&1
echo "[profile] L2 hits and misses (random order, then renumbered)" >&2
timeout -s KILL 120 rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum -f csv -d "$OUT/prof_l2" -o l2 -- \
    python3 "$ROOT/bench.py" --steps 1 --warmup 0 --fv-steps 20 --no-cpu-baseline --hbm-N 0 --skip-batch \
    > "$OUT/prof_l2.log" 2>&1
echo "[profile] done" >&2
