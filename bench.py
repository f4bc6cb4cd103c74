"""Throughput of the explicit unstructured FV Euler step on one MI355X.

One bench "step" is one whole job of the hot path on the 1024 x 1024-quad
periodic mesh (2,097,152 triangles) whose cells arrive in random order, with
the mesh and the initial state already resident in device memory:

  1. GPU Cuthill-McKee renumbering of the mesh (pseudo-peripheral search and
     breadth-first labelling) and the permutation gather of every per-cell
     array,
  2. the initial state gathered into the new order,
  3. 1000 forward-Euler Lax-Friedrichs steps (FP64),
  4. the final state gathered back to the original order (in device memory).

value = cells x 1000 / job time (cell updates per second, whole job).
Also reported: the step kernel alone (HIP events over its 1000 launches on
the library's stream) against the HBM roofline at 132 algorithmic bytes per
cell update (and at the 96 bytes of the library's compact layout), the
counter bytes per launch from the committed profile, the same kernel on a
2048 x 2048-quad mesh whose working set is beyond the Infinity Cache, the
kernel on the random (not renumbered) order, and the CPU oracle timed on a
bounded sample of the same job on every core of the host's share (and on
one core).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--fv-steps 1000]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic HBM bytes of one cell update (section 8(d) accounting of the
# path): read U 32 + neighbour ids 3 x 4 + normals 3 x 2 x 8 + 1/area 8,
# write U 32 = 132 bytes; the three neighbour states count as the cache reuse
# the renumbering provides.  `roofline.achieved` and `frac` use these bytes.
# The library stores the renumbered mesh more compactly (16-bit neighbour
# offsets, the third normal derived, two normals in 32-bit fixed point:
# 96 bytes, fv_bytes_per_update); that layout's figures are reported beside
# them (`layout_*`).
ALG_BYTES_PER_UPDATE = 132
HBM_PEAK_GBS = 8000.0
STEP_SOURCE = os.path.join(ROOT, "paper_1408_5715_amd", "csrc", "fv_step.hip")
# HBM traffic of one step launch on the 1024 x 1024 workload, measured by the
# FETCH_SIZE and WRITE_SIZE counter runs of profile.sh and written by
# profile_summary.py into this file as a `traffic-record` line, with the
# SHA-256 of the step kernel's source it was measured with.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fv_step_c2_counters.md")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha() -> str:
    with open(STEP_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(cells: int):
    """Counter bytes per step launch from TRAFFIC_FILE, or None when the file
    has no record for this mesh size or the step kernel changed since."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("source_sha256") == source_sha() and rec.get("cells") == cells:
                return rec
    return None


def cpu_threads() -> int:
    """Host threads the CPU baseline may use: OMP_NUM_THREADS when set (the
    share of the host given to this job), else the cores this process may
    run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_model() -> str:
    """The host CPU's model name with its family, model and stepping numbers
    (some hosts report only a short model name)."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" in ln:
                    k, v = (x.strip() for x in ln.split(":", 1))
                    fields.setdefault(k, v)
    except OSError:
        return ""
    name = fields.get("model name", "")
    ids = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(ids)})" if ids else name


def cpu_baseline(m, U0, dt, fv_steps: int, sample_steps: int) -> dict:
    """The oracle as it stands on this host: its Cuthill-McKee order of the
    random-order mesh (sequential code) plus sample_steps steps on the
    renumbered mesh with the cell loop on every available core, scaled to the
    job; beside it the same steps on one core, and on the random order."""
    import numpy as np

    import oracle
    from fvgen.mesh import permute_mesh

    threads = cpu_threads()
    t0 = time.perf_counter()
    perm = oracle.cm_order(m.nbr)
    t_cm = time.perf_counter() - t0
    mc = permute_mesh(m, perm.astype(np.int64))
    Uc = U0[perm]
    t0 = time.perf_counter()
    _, used = oracle.step_threads(mc.nbr, mc.nrm, mc.area, Uc, dt, sample_steps, threads)
    t_all = (time.perf_counter() - t0) / sample_steps
    one = max(2, sample_steps // 8)
    t0 = time.perf_counter()
    oracle.step(mc.nbr, mc.nrm, mc.area, Uc, dt, one)
    t_one = (time.perf_counter() - t0) / one
    # one core on the random order: the CPU side of the renumbering comparison
    # (section 7.2 measures 3-15 % on one core)
    rnd = max(1, one // 2)
    t0 = time.perf_counter()
    oracle.step(m.nbr, m.nrm, m.area, U0, dt, rnd)
    t_rnd = (time.perf_counter() - t0) / rnd
    job = t_cm + fv_steps * t_all
    return {
        "value": m.n * fv_steps / job,
        "unit": "cell-updates/s",
        "cores": used,
        "kind": "oracle",
        "sample": (f"oracle Cuthill-McKee order of the {m.n}-cell mesh ({t_cm:.2f} s, sequential) "
                   f"plus {sample_steps} oracle steps on the renumbered mesh with the cell loop "
                   f"on {used} threads ({t_all * 1e3:.1f} ms/step), scaled to the "
                   f"{fv_steps}-step job; {one} steps on one core; {rnd} on the random order"),
        "step_only_value": m.n / t_all,
        "one_core": {"value": m.n * fv_steps / (t_cm + fv_steps * t_one),
                     "step_only_value": m.n / t_one,
                     "renumbered_s_per_step": t_one,
                     "random_order_s_per_step": t_rnd},
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
    }


def hbm_resident_step(dev, N: int, fv_steps: int, snap_bits: int = 32,
                      warm_steps: int = 200) -> dict:
    """The step kernel on an N x N-quad mesh, renumbered: HIP events over
    fv_steps launches after warm_steps untimed ones.  N = 2048 (8,388,608
    cells, about 0.8 GB read and written per step) puts the working set far
    beyond the 256 MB Infinity Cache.  snap_bits > 32 gives a mesh whose
    normals are not multiples of 2^-32, so the step reads them as float64
    (the layout of a general mesh with exact vertex differences, 112 bytes
    per update).  After the renumbering, which keeps one CU busy, the first
    25-30 ms of steps run at a clock that is still settling (per launch:
    164 us, up to 198 us, then a gradual return to 167 us at 2048 x 2048);
    the warm-up covers that window so that the timed launches show the
    kernel's settled rate."""
    import torch

    import paper_1408_5715_amd as fv
    from fvgen import ic
    from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation

    log(f"step case: generating the {N}x{N}-quad mesh (coordinates on a 2^-{snap_bits} grid)")
    m = permute_mesh(periodic_mesh(N, seed=1, snap_bits=snap_bits),
                     random_permutation(2 * N * N, 2))
    P = ic.bumps_primitive(m.centroid, seed=3)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter, 0.4)
    s = fv.Solver(m.nbr, m.nrm, m.area, device=dev)
    try:
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        a, b = ev(), ev()
        a.record(s.stream)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        b.record(s.stream)
        torch.cuda.synchronize()
        renum_ms = a.elapsed_time(b)
        s.upload_state(U0)
        fv.fv_step(s.ctx, warm_steps, dt)
        a, b = ev(), ev()
        a.record(s.stream)
        fv.fv_step(s.ctx, fv_steps, dt)
        b.record(s.stream)
        torch.cuda.synchronize()
        t = a.elapsed_time(b) * 1e-3 / fv_steps
        layout = fv.fv_bytes_per_update(s.ctx)
    finally:
        s.close()
    achieved = ALG_BYTES_PER_UPDATE * m.n / t / 1e9
    return {
        "workload": (f"periodic jittered {N}x{N}-quad mesh ({m.n} cells), coordinates on a "
                     f"2^-{snap_bits} grid, renumbered on the GPU, bump state; {fv_steps} steps "
                     f"timed after {warm_steps}"),
        "warm_steps": warm_steps,
        "cells": m.n,
        "step_us": t * 1e6,
        "cell_updates_per_s": m.n / t,
        "achieved": achieved,
        "frac": achieved / HBM_PEAK_GBS,
        "layout_bytes_per_cell_update": layout,
        "layout_achieved": layout * m.n / t / 1e9,
        "renumber_ms": renum_ms,
    }


def batch_case(dev, fv_steps: int, warmup: int, reps: int) -> dict:
    """The batched workload: renumber every mesh of the 64-mesh batch (one
    workgroup each, side by side), tune the launch shape, then time fv_steps
    steps over all meshes, reps times after warmup untimed runs, with the
    tuned launch and with persistent workgroups replayed from one graph."""
    import numpy as np
    import torch

    import paper_1408_5715_amd as fv
    from fvgen.batch import batch_workload, concat
    from paper_1408_5715_amd import autotune

    log("generating the 64-mesh batch")
    parts, begin, sizes, Us, dts = batch_workload()
    nbr, nrm, area = concat(parts)
    U0 = np.concatenate(Us)
    n = int(begin[-1])
    log(f"uploading {n} cells in {len(parts)} meshes")
    s = fv.Solver(nbr, nrm, area, device=dev, mesh_begin=begin)
    dU0 = torch.from_numpy(U0).to(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    a, b = ev(), ev()
    a.record(s.stream)
    fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
    b.record(s.stream)
    torch.cuda.synchronize()
    renum_ms = a.elapsed_time(b)
    passes = s.renumber_passes()
    s.upload_state(dU0)
    tuned = autotune.tune(s, dts, steps=10)
    log(f"launch: block {tuned['block']} grid {tuned['grid']} graph {tuned['graph']}"
        f"{' (cached)' if tuned.get('cached') else ''}")

    def timed() -> float:
        times = []
        for _ in range(warmup + reps):
            s.upload_state(dU0)
            a, b = ev(), ev()
            a.record(s.stream)
            s.step(fv_steps, dts)
            b.record(s.stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return float(np.median(times[warmup:]))

    ms = timed()
    bpu = fv.fv_bytes_per_update(s.ctx)
    # the configuration's own launch form, beside the tuned one: persistent
    # workgroups (5 per CU) striding over the tiles, the whole step sequence
    # captured once into a HIP graph and replayed as one launch
    persistent = {"block": 256, "grid": 5 * torch.cuda.get_device_properties(dev).multi_processor_count,
                  "graph": True}
    s.set_launch(persistent["block"], persistent["grid"], persistent["graph"])
    pms = timed()
    persistent.update({"step_us": pms * 1e3 / fv_steps,
                       "cell_updates_per_s": n * fv_steps / (pms * 1e-3)})
    s.close()
    achieved = ALG_BYTES_PER_UPDATE * n * fv_steps / (ms * 1e-3) / 1e9
    return {
        "workload": (f"batch of {len(parts)} periodic jittered meshes "
                     f"({int(sizes.min())}..{int(sizes.max())} quads per side, "
                     f"{n} cells), {fv_steps} FP64 steps per run, per-mesh dt"),
        "cells": n, "meshes": len(parts), "fv_steps": fv_steps, "ms": ms,
        "step_us": ms * 1e3 / fv_steps,
        "cell_updates_per_s": n * fv_steps / (ms * 1e-3),
        "achieved": achieved, "frac": achieved / HBM_PEAK_GBS,
        "layout_bytes_per_cell_update": bpu,
        "layout_achieved": bpu * n * fv_steps / (ms * 1e-3) / 1e9,
        "launch": {k: tuned[k] for k in ("block", "grid", "graph")},
        "persistent_graph_launch": persistent,
        "renumber_ms": renum_ms, "renumber_passes_max": int(passes.max()),
    }


def bench_batch(args, dev) -> int:
    """The batched workload as its own line."""
    fv_steps = args.fv_steps if args.fv_steps != 1000 else 500
    c = batch_case(dev, fv_steps, args.warmup, args.steps)
    ms = c["ms"]
    rec = {
        "metric": "cell-updates/s",
        "value": c["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": c["workload"], "cells": c["cells"], "meshes": c["meshes"],
                   "fv_steps": fv_steps},
        "roofline": {"bound": "hbm", "kernel": "fv_step_kernel",
                     "achieved": c["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": c["frac"], "traffic": None,
                     "bytes_per_cell_update": ALG_BYTES_PER_UPDATE,
                     "layout_bytes_per_cell_update": c["layout_bytes_per_cell_update"],
                     "layout_achieved": c["layout_achieved"]},
        "launch": c["launch"],
        "persistent_graph_launch": c["persistent_graph_launch"],
        "breakdown": {"renumber_ms": c["renumber_ms"],
                      "renumber_passes_max": c["renumber_passes_max"],
                      "step_us": c["step_us"]},
    }
    print(json.dumps(rec), flush=True)
    return 0


def bench_hbm(args, dev) -> int:
    """The step alone on the --hbm-N mesh (the `hbm_resident` case of the
    default line) as its own line; --probe-copy runs the calibration copy
    first."""
    import torch

    if args.probe_copy:
        probe_copy(dev)
    N = args.hbm_N if args.hbm_N > 0 else 2048
    fv_steps = args.fv_steps if args.fv_steps != 1000 else 200
    c = hbm_resident_step(dev, N, fv_steps, snap_bits=args.snap_bits, warm_steps=args.hbm_warm)
    torch.cuda.synchronize()
    rec = {
        "metric": "cell-updates/s",
        "value": c["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": fv_steps,
        "warmup": c["warm_steps"],
        "ms_per_step": c["step_us"] * 1e-3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": c["workload"], "cells": c["cells"]},
        "roofline": {"bound": "hbm", "kernel": "fv_step_kernel",
                     "achieved": c["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": c["frac"], "traffic": None,
                     "bytes_per_cell_update": ALG_BYTES_PER_UPDATE,
                     "layout_bytes_per_cell_update": c["layout_bytes_per_cell_update"],
                     "layout_achieved": c["layout_achieved"]},
        "breakdown": {"renumber_ms": c["renumber_ms"], "step_us": c["step_us"]},
    }
    print(json.dumps(rec), flush=True)
    return 0


def probe_copy(dev) -> None:
    """A plain copy of known traffic (256 MiB read and 256 MiB written per
    launch, after a fill of the source) that calibrates the byte counters."""
    import torch

    src = torch.ones(32 * 2**20, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


# Useful multiply-adds of one MLP row (12 -> 64 -> 64 -> 4); a cell evaluates
# 6 rows (3 faces, both orientations).
MLP_FLOPS_PER_CELL = 6 * 2 * (12 * 64 + 64 * 64 + 64 * 4)
BF16_PEAK_TFLOPS = 2500.0


def bench_learned(args, dev) -> int:
    """The learned-correction comparison: the corrected coarse solver
    (1024 x 1024 quads) against the plain coarse one, the plain fine one
    (2048 x 2048) and a plain 4096 x 4096 reference, all from the same seeded
    flow: L2 density errors against the reference after 64, 256 and 2000
    coarse steps, and the step rate of each solver."""
    from paper_1408_5715_amd import learned

    N = args.N
    steps = 2000 if args.fv_steps == 1000 else args.fv_steps
    seeds = [5000]
    p = learned.load_params()
    horizons = sorted({64, 256, steps})
    lv = learned.compare_levels(p, N, seeds, horizons)
    timing = learned.compare(p, N, 2, seeds, 64, timing_steps=200)
    cc = timing["coarse_corrected"]["cell_updates_per_s"]
    fp = timing["fine_plain"]["cell_updates_per_s"]
    cp = timing["coarse_plain"]["cell_updates_per_s"]
    t_coarse = steps / (cc / timing["coarse_cells"])
    t_fine = 2 * steps / (fp / timing["fine_cells"])
    achieved = MLP_FLOPS_PER_CELL * cc / 1e12
    errs, vs_fine = {}, {}
    for r in lv["flows"]:
        gap = r["coarse_plain"] - r["fine_plain"]
        errs[str(r["steps"])] = {k: r[k] for k in ("coarse_plain", "coarse_corrected",
                                                    "fine_plain")}
        vs_fine[str(r["steps"])] = {"coarse_plain": r["coarse_plain_vs_fine"],
                                    "coarse_corrected": r["coarse_corrected_vs_fine"]}
        errs[str(r["steps"])]["gap_closed"] = (r["coarse_plain"] - r["coarse_corrected"]) / gap
    rec = {
        "metric": "learned vs plain at equal L2 density error",
        "value": cc,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": timing["coarse_corrected"]["us_per_step"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 flux and update, bf16 MLP with f32 accumulation",
        "data": "synthetic",
        "config": {"workload": (f"learned-corrected {N}x{N}-quad coarse mesh vs plain "
                                f"{2 * N}x{2 * N} fine mesh (unjittered, nested), errors against a "
                                f"plain {4 * N}x{4 * N} reference after up to {steps} coarse "
                                f"steps, seeded vortex + bump flow {seeds}"),
                   "coarse_cells": timing["coarse_cells"], "fine_cells": timing["fine_cells"],
                   "coarse_steps": steps, "dt_coarse": timing["dt_coarse"]},
        "roofline": {"bound": "mfma", "kernel": "fv_step_learned_kernel", "achieved": achieved,
                     "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                     "flops_per_cell_update": MLP_FLOPS_PER_CELL},
        "cpu_baseline": None,
        "comparison": {
            "fine_plain_cell_updates_per_s": fp,
            "coarse_plain_cell_updates_per_s": cp,
            "time_to_solution_fine_over_coarse_corrected": t_fine / t_coarse,
            "l2_rho_vs_reference": errs,
            # the same coarse solutions against the restricted plain
            # 2N x 2N solution itself
            "l2_rho_vs_fine_plain": vs_fine,
        },
    }
    print(json.dumps(rec), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed jobs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed jobs")
    ap.add_argument("--fv-steps", type=int, default=1000, help="time steps per job")
    ap.add_argument("--N", type=int, default=1024, help="quads per side")
    ap.add_argument("--cpu-sample-steps", type=int, default=200,
                    help="oracle steps of the all-core CPU sample (one core runs 1/8 of them)")
    ap.add_argument("--hbm-N", type=int, default=2048,
                    help="quads per side of the HBM-resident step timing (0: skip)")
    ap.add_argument("--hbm-warm", type=int, default=200,
                    help="untimed steps before the timed ones of --workload hbm")
    ap.add_argument("--snap-bits", type=int, default=32,
                    help="--workload hbm: coordinates on a 2^-bits grid (32: the compact "
                         "96-byte layout; 40: float64 normals, 112 bytes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-batch", action="store_true",
                    help="leave the 64-mesh batch case out of the default line")
    ap.add_argument("--skip-random", action="store_true",
                    help="skip timing the step on the random (not renumbered) order")
    ap.add_argument("--workload", choices=("single", "batch", "learned", "hbm"),
                    default="single",
                    help="single: the 1024x1024-quad job (default line); batch: 64 meshes of "
                         "20k-500k cells advanced together; learned: the corrected 1024x1024 "
                         "solver against the plain 1024x1024 and 2048x2048 ones and a "
                         "4096x4096 reference; hbm: the step alone on the --hbm-N mesh "
                         "(default 2048x2048, beyond the Infinity Cache)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the step would shard by contiguous ranges of the renumbered order with a "
              "halo exchange per step; that exchange is not implemented).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1408_5715_amd as fv
    from fvgen import ic
    from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch":
        return bench_batch(args, dev)
    if args.workload == "learned":
        return bench_learned(args, dev)
    if args.workload == "hbm":
        return bench_hbm(args, dev)

    N = args.N
    log(f"generating the {N}x{N}-quad mesh")
    m = permute_mesh(periodic_mesh(N, seed=1), random_permutation(2 * N * N, 2))
    P = ic.bumps_primitive(m.centroid, seed=3)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter, 0.4)
    n = m.n

    log("uploading")
    s = fv.Solver(m.nbr, m.nrm, m.area, device=dev)
    stream = s.stream
    dU0 = torch.from_numpy(U0).to(dev)
    dout = torch.empty_like(dU0)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    half = args.fv_steps // 2

    def job(record=None):
        e0, e1, eh, e2, e3 = ev(), ev(), ev(), ev(), ev()
        e0.record(stream)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        fv.fv_upload_state_device(s.ctx, dU0)
        e1.record(stream)
        # the same steps in two calls, with an event between the halves
        fv.fv_step(s.ctx, half, dt)
        eh.record(stream)
        fv.fv_step(s.ctx, args.fv_steps - half, dt)
        e2.record(stream)
        fv.fv_download_state_device(s.ctx, dout)
        e3.record(stream)
        if record is not None:
            record.append((e0, e1, e2, e3, eh))

    log(f"warmup: {args.warmup} job(s)")
    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()

    log(f"timing {args.steps} job(s) of {args.fv_steps} steps")
    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        job(marks)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    layout_bytes = fv.fv_bytes_per_update(s.ctx)
    renum_ms = [a.elapsed_time(b) for a, b, _, _, _ in marks]
    step_ms = [b.elapsed_time(c) for _, b, c, _, _ in marks]
    first_half_ms = [b.elapsed_time(h) for _, b, _, _, h in marks]
    second_half_ms = [h.elapsed_time(c) for _, _, c, _, h in marks]
    down_ms = [c.elapsed_time(d) for _, _, c, d, _ in marks]
    ms_per_job = wall * 1e3 / args.steps
    value = n * args.fv_steps * args.steps / wall
    step_kernel_s = float(np.mean(step_ms)) * 1e-3 / args.fv_steps
    achieved = ALG_BYTES_PER_UPDATE * n / step_kernel_s / 1e9

    # the same kernel on the random (identity) order, for the locality effect
    random_step_s = float("nan")
    random_bytes_per_update = None
    if not args.skip_random:
        log("timing the step on the random order")
        fv.fv_renumber(s.ctx, fv.FV_ORDER_IDENTITY)
        random_bytes_per_update = fv.fv_bytes_per_update(s.ctx)
        fv.fv_upload_state_device(s.ctx, dU0)
        fv.fv_step(s.ctx, 50, dt)
        a, b = ev(), ev()
        a.record(stream)
        fv.fv_step(s.ctx, args.fv_steps, dt)
        b.record(stream)
        torch.cuda.synchronize()
        random_step_s = a.elapsed_time(b) * 1e-3 / args.fv_steps
    s.close()
    del dU0, dout

    if args.probe_copy:
        probe_copy(dev)

    hbm = None
    general = None
    general_hbm = None
    if args.hbm_N > 0:
        hbm = hbm_resident_step(dev, args.hbm_N, 200, warm_steps=200)
        general = hbm_resident_step(dev, N, 400, snap_bits=40, warm_steps=800)
        general_hbm = hbm_resident_step(dev, args.hbm_N, 200, snap_bits=40, warm_steps=200)
        torch.cuda.empty_cache()
    batch = None
    if not args.skip_batch:
        batch = batch_case(dev, 500, 1, 3)
        torch.cuda.empty_cache()

    trec = measured_traffic(n)
    traffic = None if trec is None else trec["fetch_bytes"] + trec["write_bytes"]

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline ({args.cpu_sample_steps} steps + CM order)")
        cpu = cpu_baseline(m, U0, dt, args.fv_steps, args.cpu_sample_steps)

    rec = {
        "metric": "cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_job,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"periodic jittered {N}x{N}-quad triangle mesh ({n} cells), random cell "
                         f"order, Mach 0.5 stream + 32 bumps, CFL 0.4; job = GPU Cuthill-McKee "
                         f"renumbering + gather + {args.fv_steps} FP64 Lax-Friedrichs steps + "
                         f"gather back"),
            "cells": n,
            "fv_steps_per_job": args.fv_steps,
            "dt": dt,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "fv_step_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_source": None if trec is None else os.path.relpath(TRAFFIC_FILE, ROOT),
            "bytes_per_cell_update": ALG_BYTES_PER_UPDATE,
            "avg_launch_us": step_kernel_s * 1e6,
            "layout_bytes_per_cell_update": layout_bytes,
            "layout_achieved": layout_bytes * n / step_kernel_s / 1e9,
            "layout_frac": layout_bytes * n / step_kernel_s / 1e9 / HBM_PEAK_GBS,
            "note": ("the 1024x1024 working set (about 200 MB) fits in the 256 MB Infinity Cache; "
                     "hbm_resident times the same kernel on a mesh beyond it"),
        },
        "hbm_resident": hbm,
        # the same kernel on the same mesh snapped to a finer grid, so that
        # the two stored normals stay float64 (the general-mesh layout)
        "general_layout": general,
        # ... and on the mesh beyond the Infinity Cache
        "general_layout_hbm_resident": general_hbm,
        # the 64-mesh batch (20k..500k cells each, 11.9M in all), 500 steps
        "batch": batch,
        "cpu_baseline": cpu,
        "breakdown": {
            "renumber_and_upload_ms": float(np.median(renum_ms)),
            "steps_ms": float(np.median(step_ms)),
            # the job's steps split in halves: the first half includes the
            # slow-down that follows the renumbering's near-idle chip
            "first_half_step_us": (float(np.median(first_half_ms)) * 1e3 / half
                                   if half else None),
            "second_half_step_us": float(np.median(second_half_ms)) * 1e3 / (args.fv_steps - half),
            "download_ms": float(np.median(down_ms)),
            "step_only_cell_updates_per_s": n / step_kernel_s,
            "random_order_step_us": None if args.skip_random else random_step_s * 1e6,
            "random_order_cell_updates_per_s": None if args.skip_random else n / random_step_s,
            "random_order_bytes_per_cell_update": random_bytes_per_update,
        },
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
