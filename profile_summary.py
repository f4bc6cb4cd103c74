"""Summarise the rocprofv3 output of profile.sh as Markdown.

Reads prof_trace (kernel trace + stats), prof_fetch and prof_write
(FETCH_SIZE / WRITE_SIZE per dispatch) under $FV_PROFILE_DIR (default:
profile_out/ at the repository root), as profile.sh writes them.  Byte
counters are scaled by what they read for the plain copy kernel in the same
run (256 MiB read and 256 MiB written per launch).
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics as st
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
OUT = os.environ.get("FV_PROFILE_DIR", os.path.join(ROOT, "profile_out"))
COPY_BYTES = 256 * 2**20
CELLS = 2097152
SIMDS = 1024  # 256 CUs x 4; SQ_VALU_MFMA_BUSY_CYCLES sums over them
XCDS = 8  # GRBM_GUI_ACTIVE sums over the XCDs


def short(name: str) -> str:
    name = name.replace("fvk::(anonymous namespace)::", "")
    if "elementwise" in name:
        return ("torch elementwise copy (mul by 1)" if "MulFunctor" in name or "mul" in name.lower()
                else "torch elementwise " + name.split("<")[1].split(",")[1].strip()
                if "<" in name else "torch elementwise")
    return name.split("(")[0]


def counters(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    out = {}
    for r in rows:
        out.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def trace_table(prefix: str) -> list[str]:
    """Per-kernel statistics of the kernel trace run."""
    lines = []
    stats = list(csv.DictReader(open(os.path.join(OUT, f"{prefix}_trace",
                                                  "trace_kernel_stats.csv"))))
    lines.append("| kernel | calls | avg us | min us | max us | share |")
    lines.append("|---|---|---|---|---|---|")
    for r in stats:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.1f}% |")
    return lines


def byte_table(prefix: str, cells: int):
    """FETCH_SIZE / WRITE_SIZE per launch, scaled by the copy kernel's
    readings; returns the lines and the step kernel's (fetch, write) bytes."""
    lines = []
    f = counters(os.path.join(OUT, f"{prefix}_fetch", "fetch_counter_collection.csv"),
                 "FETCH_SIZE")
    w = counters(os.path.join(OUT, f"{prefix}_write", "write_counter_collection.csv"),
                 "WRITE_SIZE")
    copy = "torch elementwise copy (mul by 1)"
    # the first elementwise launch is the fill of the source (no read)
    fcopy = st.mean(f[copy][1:]) * 1024
    wcopy = st.mean(w[copy]) * 1024
    fs, ws = COPY_BYTES / fcopy, COPY_BYTES / wcopy
    lines.append(f"Copy calibration: FETCH_SIZE reads {fcopy / 2**20:.1f} MiB and WRITE_SIZE "
                 f"{wcopy / 2**20:.1f} MiB for 256 MiB each; scale factors {fs:.3f} and {ws:.3f}.")
    lines.append("")
    lines.append("| kernel | launches | FETCH MiB/launch (scaled) | WRITE MiB/launch (scaled) | "
                 "bytes/cell (scaled) |")
    lines.append("|---|---|---|---|---|")
    step = None
    for k in sorted(f):
        if k == copy or k not in w:
            continue
        fb = st.mean(f[k]) * 1024 * fs
        wb = st.mean(w[k]) * 1024 * ws
        lines.append(f"| {k} | {len(f[k])} | {fb / 2**20:.1f} | {wb / 2**20:.1f} | "
                     f"{(fb + wb) / cells:.1f} |")
        if "fv_step_kernel" in k:
            step = (round(fb), round(wb))
    if step:
        lines.append("")
        lines.append(f"fv_step_kernel per launch (scaled): fetch {step[0]:,} B + write {step[1]:,} B "
                     f"= {step[0] + step[1]:,} B")
    return lines, step, (fs, ws)


def main() -> int:
    lines = trace_table("prof")
    lines.append("")
    table, step, (fs, ws) = byte_table("prof", CELLS)
    lines += table
    if step:
        # machine-readable line bench.py reads as its `traffic`, valid for the
        # step kernel source it was measured with
        with open(os.path.join(ROOT, "paper_1408_5715_amd", "csrc", "fv_step.hip"), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
        lines.append("")
        lines.append("traffic-record: " + json.dumps(
            {"kernel": "fv_step_kernel", "cells": CELLS, "source_sha256": sha,
             "fetch_bytes": step[0], "write_bytes": step[1],
             "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)}))
    l2 = os.path.join(OUT, "prof_l2", "l2_counter_collection.csv")
    if os.path.exists(l2):
        hit = counters(l2, "TCC_HIT_sum")
        miss = counters(l2, "TCC_MISS_sum")
        lines.append("")
        lines.append("| step kernel variant | launches | L2 hits / launch | L2 misses / launch | "
                     "L2 hit rate |")
        lines.append("|---|---|---|---|---|")
        for k in sorted(hit):
            if "fv_step_kernel" in k and k in miss:
                h, m = st.mean(hit[k]), st.mean(miss[k])
                lines.append(f"| {k} | {len(hit[k])} | {h:.4g} | {m:.4g} | {h / (h + m):.3f} |")
    log = os.path.join(OUT, "prof_trace.log")
    if os.path.exists(log):
        for line in open(log):
            if line.startswith("{"):
                lines.append("")
                lines.append("bench.py line of the traced run: `" + line.strip() + "`")
    print("\n".join(lines))
    return 0


def main_hbm() -> int:
    """profile.sh hbm: the step on the 2048 x 2048-quad mesh."""
    cells = 2 * 2048 * 2048
    lines = trace_table("hprof")
    table, step, _ = byte_table("hprof", cells)
    # the step's launches in order: the warm-up ones, then the timed ones
    path = os.path.join(OUT, "hprof_trace", "trace_kernel_trace.csv")
    rows = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                  for r in csv.DictReader(open(path)) if "fv_step_kernel" in r["Kernel_Name"])
    us = [(e - b) / 1e3 for b, e in rows]
    if len(us) >= 40 and step:
        moved = step[0] + step[1]
        lines.append("")
        lines.append("fv_step_kernel launches in order, mean us per block of 20: "
                     + ", ".join(f"{st.mean(us[i:i + 20]):.1f}" for i in range(0, len(us), 20)))
        half = len(us) // 2
        lines.append("")
        lines.append(f"fv_step_kernel: first {half} launches {st.mean(us[:half]):.2f} us, "
                     f"last {len(us) - half} launches {st.mean(us[half:]):.2f} us "
                     f"({moved / st.mean(us[half:]) / 1e3:.0f} GB/s at the measured "
                     f"{moved / cells:.1f} B per cell)")
    lines.append("")
    lines += table
    for name in ("hprof_trace.log", "hprof_fetch.log"):
        log = os.path.join(OUT, name)
        if os.path.exists(log):
            for line in open(log):
                if line.startswith("{"):
                    lines.append("")
                    lines.append(f"bench.py line of the {name.split('_')[1].split('.')[0]} run: `"
                                 + line.strip() + "`")
    print("\n".join(lines))
    return 0


def main_orders() -> int:
    """Summary of `profile.sh orders`: the step launches of the comparison
    come as runs of 20 + 150 (random), 20 + 200 (AM1) and 20 + 250
    (Cuthill-McKee) launches, in that order (tests/test_gpu_irregular.py
    COMMON and RUNS)."""
    path = os.path.join(OUT, "oprof_l2", "l2_counter_collection.csv")
    rows = [r for r in csv.DictReader(open(path)) if "fv_step_kernel" in r["Kernel_Name"]]
    per = {}
    for r in rows:
        d = per.setdefault(int(r["Dispatch_Id"]), {"name": short(r["Kernel_Name"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    ids = sorted(per)
    lines = ["| order | step launches | kernel | L2 hits / launch | L2 misses / launch | L2 hit rate |",
             "|---|---|---|---|---|---|"]
    k = 0
    for name, count in (("random", 170), ("AM1", 220), ("Cuthill-McKee", 270)):
        run = [per[i] for i in ids[k:k + count]]
        k += count
        h = st.mean(d["TCC_HIT_sum"] for d in run)
        m = st.mean(d["TCC_MISS_sum"] for d in run)
        lines.append(f"| {name} | {len(run)} | {run[0]['name']} | {h:.4g} | {m:.4g} | "
                     f"{h / (h + m):.3f} |")
    log = os.path.join(OUT, "oprof_l2.log")
    if os.path.exists(log):
        lines.append("")
        lines += [ln.rstrip() for ln in open(log) if ln.startswith("irregular")]
    print("\n".join(lines))
    return 0


def main_learned() -> int:
    """Summary of `profile.sh learned`."""
    lines = []
    stats = list(csv.DictReader(open(os.path.join(OUT, "lprof_trace", "trace_kernel_stats.csv"))))
    lines.append("| kernel | calls | avg us | min us | max us | share |")
    lines.append("|---|---|---|---|---|---|")
    for r in stats:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.1f}% |")
    for line in open(os.path.join(OUT, "lprof_trace.log")):
        if line.startswith("corrected"):
            lines.append("")
            lines.append("Same process, HIP events: " + line.strip())
    path = os.path.join(OUT, "lprof_mfma", "mfma_counter_collection.csv")
    per = {}
    for r in csv.DictReader(open(path)):
        per.setdefault(short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
            float(r["Counter_Value"]))
    lines.append("")
    lines.append("| kernel | launches | waves | MFMA / wave | other VALU / wave | LDS / wave | "
                 "bf16 MFMA flop / launch | MFMA busy cycles per SIMD / GPU cycles |")
    lines.append("|---|---|---|---|---|---|---|---|")
    for k in sorted(per):
        c = {n: st.mean(v) for n, v in per[k].items()}
        if not c.get("SQ_INSTS_MFMA"):
            continue
        w = c["SQ_WAVES"]
        lines.append(f"| {k} | {len(per[k]['SQ_WAVES'])} | {w:.0f} | {c['SQ_INSTS_MFMA'] / w:.0f} | "
                     f"{(c['SQ_INSTS_VALU'] - c['SQ_INSTS_MFMA']) / w:.0f} | "
                     f"{c['SQ_INSTS_LDS'] / w:.0f} | {c['SQ_INSTS_VALU_MFMA_MOPS_BF16'] * 512:.4g} | "
                     f"{(c['SQ_VALU_MFMA_BUSY_CYCLES'] / SIMDS) / (c['GRBM_GUI_ACTIVE'] / XCDS):.2f} |")
    f = counters(os.path.join(OUT, "lprof_fetch", "fetch_counter_collection.csv"), "FETCH_SIZE")
    copy = "torch elementwise copy (mul by 1)"
    if copy in f:
        fcopy = st.mean(f[copy][1:] if len(f[copy]) > 1 else f[copy]) * 1024
        fs = COPY_BYTES / fcopy
        lines.append("")
        lines.append(f"FETCH_SIZE of the 256 MiB copy in the same run: {fcopy / 2**20:.1f} MiB "
                     f"(scale x{fs:.3f}).")
        for k in sorted(f):
            if "learned" in k:
                fb = st.mean(f[k]) * 1024 * fs
                lines.append(f"{k}: {fb / 2**20:.1f} MiB fetched per launch (scaled), "
                             f"{fb / CELLS:.1f} B per cell")
    print("\n".join(lines))
    return 0


def per_dispatch(path):
    """{kernel: {counter: mean value per dispatch}} of a counter run."""
    agg = {}
    for r in csv.DictReader(open(path)):
        agg.setdefault(short(r["Kernel_Name"]), {}).setdefault(r["Counter_Name"], []).append(
            float(r["Counter_Value"]))
    return {k: {c: st.mean(v) for c, v in d.items()} for k, d in agg.items()}


def main_renumber() -> int:
    """Counters of the renumbering kernels and the step (profile.sh renumber).
    SQ cycle counters are in units of 4 cycles; TA and TCP counters sum over
    the CUs (one CU for a renumbering kernel, all 256 for the step)."""
    sq = per_dispatch(os.path.join(OUT, "rprof_sq", "sq_counter_collection.csv"))
    mem = per_dispatch(os.path.join(OUT, "rprof_mem", "mem_counter_collection.csv"))
    # the compact step (renumbered order, 16-bit offsets, fixed-point normals)
    step = next((k for k in sq if k.startswith("void fv_step_kernel<256, true, true, true")),
                "void fv_step_kernel<256, true, true, true, false>")
    # (kernel, CUs it runs on, levels it walks): the labelling pass and the
    # confirming sweep run on one CU each
    rows = [("cm_first_kernel", 1, 1366),
            ("cm_rename_kernel", 256, 0), ("cm_probe_kernel", 1, 1366),
            ("cm_finish_kernel", 1, 0), (step, 256, 0)]
    lines = ["| kernel | cycles | waves | VALU / wave | VMEM reads / wave | VALU busy / SIMD "
             "| waves waiting: any / on data | TA busy / stalled by L1 | L1->L2 reads "
             "| L2 read latency (cycles) |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for k, cus, levels in rows:
        if k not in sq or k not in mem:
            continue
        q, m = sq[k], mem[k]
        cycles = m["GRBM_GUI_ACTIVE"] / XCDS
        waves = q["SQ_WAVES"]
        valu_busy = q["SQ_ACTIVE_INST_VALU"] * 4 / (cus * 4 * cycles)
        lines.append(
            f"| {k} | {cycles:.3g} | {waves:.0f} | {q['SQ_INSTS_VALU'] / waves:.0f} | "
            f"{q['SQ_INSTS_VMEM_RD'] / waves:.1f} | {valu_busy:.2f} | "
            f"{q['SQ_WAIT_ANY'] / q['SQ_WAVE_CYCLES']:.2f} / "
            f"{q['SQ_WAIT_INST_ANY'] / q['SQ_WAVE_CYCLES']:.2f} | "
            f"{m['TA_TA_BUSY'] / (cus * cycles):.2f} / "
            f"{m['TA_ADDR_STALLED_BY_TC_CYCLES'] / (cus * cycles):.2f} | "
            f"{m['TCP_TCC_READ_REQ']:.3g} | "
            f"{m['TCP_TCC_READ_REQ_LATENCY'] / max(m['TCP_TCC_READ_REQ'], 1):.0f} |")
        if levels:
            lines.append(f"| (per level) | {cycles / levels:.0f} | | "
                         f"{q['SQ_INSTS_VALU'] / waves / levels:.0f} | "
                         f"{q['SQ_INSTS_VMEM_RD'] / waves / levels:.1f} | | | | "
                         f"{m['TCP_TCC_READ_REQ'] / levels:.0f} | |")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "learned":
        sys.exit(main_learned())
    if len(sys.argv) > 1 and sys.argv[1] == "hbm":
        sys.exit(main_hbm())
    if len(sys.argv) > 1 and sys.argv[1] == "orders":
        sys.exit(main_orders())
    if len(sys.argv) > 1 and sys.argv[1] == "renumber":
        sys.exit(main_renumber())
    sys.exit(main())
