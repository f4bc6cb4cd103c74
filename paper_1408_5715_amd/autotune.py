"""Launch-shape autotuner for the step kernel.

Times every candidate (workgroup size x grid x graph capture) on the
solver's own data with HIP events and keeps the fastest.  Results are cached
as JSON, keyed by the cell count, the number of meshes, the geometry layout
(bytes per cell update) and the device name, so a later run on the same
workload skips the search.  The launch shape never changes results (bitwise),
only speed.
"""

from __future__ import annotations

import json
import os
from itertools import product

from .fvgpu import fv_bytes_per_update

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fvgpu_autotune.json")

BLOCKS = (128, 256, 512)
# 0: one workgroup per tile; otherwise persistent workgroups (multiples of the 256 CUs)
GRIDS = (0, 256, 512, 1024, 2048, 4096)


def _key(solver) -> str:
    import torch

    name = torch.cuda.get_device_name(solver.device)
    return f"{name}|cells={solver.n}|meshes={solver.n_meshes}|bytes={fv_bytes_per_update(solver.ctx)}"


def _time(solver, dt, steps: int) -> float:
    import torch

    st = solver.stream
    solver.step(2, dt)  # warm-up (and graph capture when enabled)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    solver.step(steps, dt)
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune(solver, dt, steps: int = 20, cache_path: str | None = None, force: bool = False,
         graphs=(False, True)) -> dict:
    """Pick and apply the fastest launch shape; returns the chosen entry.

    The state is advanced while timing, so call this on a scratch state (or
    upload the initial state again afterwards)."""
    path = cache_path or os.environ.get("FVGPU_TUNE_CACHE", DEFAULT_CACHE)
    key = _key(solver)
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        best = cache[key]
        solver.set_launch(best["block"], best["grid"], best["graph"])
        return dict(best, cached=True)
    trials = []
    for block, grid, graph in product(BLOCKS, GRIDS, graphs):
        solver.set_launch(block, grid, graph)
        trials.append({"block": block, "grid": grid, "graph": bool(graph),
                       "ms_per_step": _time(solver, dt, steps)})
    best = min(trials, key=lambda t: t["ms_per_step"])
    entry = dict(best, trials=trials)
    cache[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass  # a read-only home still gets the tuned launch for this process
    solver.set_launch(best["block"], best["grid"], best["graph"])
    return dict(entry, cached=False)
