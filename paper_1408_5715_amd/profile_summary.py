"""Summarise the rocprofv3 output of profile.sh as Markdown.

Reads gpurun_out/prof_trace (kernel trace + stats), gpurun_out/prof_fetch
and gpurun_out/prof_write (FETCH_SIZE / WRITE_SIZE per dispatch).  Byte
counters are scaled by what they read for the plain copy kernel in the same
run (256 MiB read and 256 MiB written per launch).
"""

from __future__ import annotations

import csv
import os
import statistics as st
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "gpurun_out")
COPY_BYTES = 256 * 2**20
CELLS = 2097152


def short(name: str) -> str:
    name = name.replace("fvk::(anonymous namespace)::", "")
    return name.split("(")[0] if "elementwise" not in name else "torch elementwise copy (mul by 1)"


def counters(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    out = {}
    for r in rows:
        out.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def main() -> int:
    lines = []
    stats = list(csv.DictReader(open(os.path.join(OUT, "prof_trace", "trace_kernel_stats.csv"))))
    lines.append("| kernel | calls | avg us | min us | max us | share |")
    lines.append("|---|---|---|---|---|---|")
    for r in stats:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.1f}% |")
    f = counters(os.path.join(OUT, "prof_fetch", "fetch_counter_collection.csv"), "FETCH_SIZE")
    w = counters(os.path.join(OUT, "prof_write", "write_counter_collection.csv"), "WRITE_SIZE")
    copy = "torch elementwise copy (mul by 1)"
    # the first elementwise launch is the fill of the source (no read)
    fcopy = st.mean(f[copy][1:]) * 1024
    wcopy = st.mean(w[copy]) * 1024
    fs, ws = COPY_BYTES / fcopy, COPY_BYTES / wcopy
    lines.append("")
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
                     f"{(fb + wb) / CELLS:.1f} |")
        if "fv_step_kernel" in k:
            step = (round(fb), round(wb))
    if step:
        lines.append("")
        lines.append(f"fv_step_kernel per launch (scaled): fetch {step[0]:,} B + write {step[1]:,} B "
                     f"= {step[0] + step[1]:,} B")
    log = os.path.join(OUT, "prof_trace.log")
    if os.path.exists(log):
        for line in open(log):
            if line.startswith("{"):
                lines.append("")
                lines.append("bench.py line of the traced run: `" + line.strip() + "`")
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
