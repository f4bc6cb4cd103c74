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
the library's stream) against the HBM roofline, the same kernel on the
random (not renumbered) order, and the CPU oracle timed on a bounded sample
of the same job.

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

# Algorithmic HBM bytes of one cell update come from the library
# (fv_bytes_per_update): each per-cell array touched once, the three
# neighbour states counted as the cache reuse the renumbering provides.
# General layout: read U 32 + neighbour ids 12 + normals 48 + 1/area 8,
# write U 32 = 132; with 16-bit neighbour offsets and the derived third
# normal 112; with, in addition, the two stored normals in 32-bit fixed point
# (the layout of this workload after renumbering) 96.
HBM_PEAK_GBS = 8000.0
STEP_SOURCE = os.path.join(ROOT, "paper_1408_5715_amd", "csrc", "fv_step.hip")

# HBM traffic of one step launch on this workload (renumbered order, 96-byte
# layout), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs, each scaled
# by what the counter reads for a plain 256 MiB copy in the same run (x2.000
# and x1.000).  Valid only for the step kernel source with this SHA-256.
MEASURED_TRAFFIC = {
    "source_sha": "02f9e3bbb22d696456438d6eaa9d030eb978559f05820e45870a06d81af9a197",
    "cells": 2097152,
    "bytes_per_launch": 202403534,  # fetch 135,295,762 + write 67,107,772
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_sha() -> str:
    with open(STEP_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def cpu_baseline(m, U0, dt, fv_steps: int, sample_steps: int) -> dict:
    """The oracle as it stands, single-threaded: CM order of the random-order
    mesh plus sample_steps steps on the renumbered mesh, scaled to the job."""
    import numpy as np

    import oracle
    from fvgen.mesh import permute_mesh

    t0 = time.perf_counter()
    perm = oracle.cm_order(m.nbr)
    t_cm = time.perf_counter() - t0
    mc = permute_mesh(m, perm.astype(np.int64))
    Uc = U0[perm]
    t0 = time.perf_counter()
    oracle.step(mc.nbr, mc.nrm, mc.area, Uc, dt, sample_steps)
    t_step = (time.perf_counter() - t0) / sample_steps
    # the same steps on the random order: the CPU side of the renumbering
    # comparison (section 7.2 measures 3-15 % on one core)
    rnd = max(1, sample_steps // 4)
    t0 = time.perf_counter()
    oracle.step(m.nbr, m.nrm, m.area, U0, dt, rnd)
    t_rnd = (time.perf_counter() - t0) / rnd
    job = t_cm + fv_steps * t_step
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                             "")
    except OSError:
        pass
    return {
        "value": m.n * fv_steps / job,
        "unit": "cell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle Cuthill-McKee order of the {m.n}-cell mesh ({t_cm:.2f} s) plus "
                   f"{sample_steps} oracle steps on the renumbered mesh ({t_step:.3f} s/step), "
                   f"scaled to the {fv_steps}-step job"),
        "step_only_value": m.n / t_step,
        "random_order_s_per_step": t_rnd,
        "renumbered_s_per_step": t_step,
        "cpu_model": cpu_model,
    }


def bench_batch(args, dev) -> int:
    """The batched workload: renumber every mesh (one workgroup each, side by
    side), tune the launch shape, then time the step over all meshes."""
    import numpy as np
    import torch

    import paper_1408_5715_amd as fv
    from fvgen.batch import batch_workload, concat
    from paper_1408_5715_amd import autotune

    fv_steps = args.fv_steps if args.fv_steps != 1000 else 500
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
    times = []
    for _ in range(args.warmup + args.steps):
        s.upload_state(dU0)
        a, b = ev(), ev()
        a.record(s.stream)
        s.step(fv_steps, dts)
        b.record(s.stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times = times[args.warmup:]
    ms = float(np.median(times))
    bpu = fv.fv_bytes_per_update(s.ctx)
    s.close()
    rec = {
        "metric": "cell-updates/s",
        "value": n * fv_steps / (ms * 1e-3),
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
        "config": {"workload": (f"batch of {len(parts)} periodic jittered meshes "
                                f"({int(sizes.min())}..{int(sizes.max())} quads per side, "
                                f"{n} cells), {fv_steps} FP64 steps per run, per-mesh dt"),
                   "cells": n, "meshes": len(parts), "fv_steps": fv_steps},
        "roofline": {"bound": "hbm", "kernel": "fv_step_kernel",
                     "achieved": bpu * n * fv_steps / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": bpu * n * fv_steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_cell_update": bpu},
        "launch": {k: tuned[k] for k in ("block", "grid", "graph")},
        "breakdown": {"renumber_ms": renum_ms, "renumber_passes_max": int(passes.max()),
                      "step_us": ms * 1e3 / fv_steps},
    }
    print(json.dumps(rec), flush=True)
    return 0


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
    errs = {}
    for r in lv["flows"]:
        gap = r["coarse_plain"] - r["fine_plain"]
        errs[str(r["steps"])] = {k: r[k] for k in ("coarse_plain", "coarse_corrected",
                                                    "fine_plain")}
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
    ap.add_argument("--cpu-sample-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-random", action="store_true",
                    help="skip timing the step on the random (not renumbered) order")
    ap.add_argument("--workload", choices=("single", "batch", "learned"), default="single",
                    help="single: the 1024x1024-quad job (default line); batch: 64 meshes of "
                         "20k-500k cells advanced together; learned: the corrected 1024x1024 "
                         "solver against the plain 1024x1024 and 2048x2048 ones and a "
                         "4096x4096 reference")
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

    def job(record=None):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record(stream)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        fv.fv_upload_state_device(s.ctx, dU0)
        e1.record(stream)
        fv.fv_step(s.ctx, args.fv_steps, dt)
        e2.record(stream)
        fv.fv_download_state_device(s.ctx, dout)
        e3.record(stream)
        if record is not None:
            record.append((e0, e1, e2, e3))

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

    bytes_per_update = fv.fv_bytes_per_update(s.ctx)
    renum_ms = [a.elapsed_time(b) for a, b, _, _ in marks]
    step_ms = [b.elapsed_time(c) for _, b, c, _ in marks]
    down_ms = [c.elapsed_time(d) for _, _, c, d in marks]
    ms_per_job = wall * 1e3 / args.steps
    value = n * args.fv_steps * args.steps / wall
    step_kernel_s = float(np.mean(step_ms)) * 1e-3 / args.fv_steps
    achieved = bytes_per_update * n / step_kernel_s / 1e9

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

    if args.probe_copy:
        # known traffic: 256 MiB read and 256 MiB written per launch
        src = torch.ones(32 * 2**20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()

    traffic = None
    if MEASURED_TRAFFIC is not None and MEASURED_TRAFFIC.get("source_sha") == source_sha() \
            and MEASURED_TRAFFIC.get("cells") == n:
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]

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
            "bytes_per_cell_update": bytes_per_update,
            "avg_launch_us": step_kernel_s * 1e6,
        },
        "cpu_baseline": cpu,
        "breakdown": {
            "renumber_and_upload_ms": float(np.median(renum_ms)),
            "steps_ms": float(np.median(step_ms)),
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
