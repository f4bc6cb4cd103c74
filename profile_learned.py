"""A short run of the learned-correction kernels for rocprofv3 (few
dispatches, so counter passes stay quick): the corrected step on the
1024 x 1024-quad C5 mesh (20 steps, after 200 warm-up steps) and, with
--adjoint, 4 corrected adjoint steps on the C4 training batch (32 flows of
128 x 128 quads) with parameter gradients."""

from __future__ import annotations

import argparse
import sys

import numpy as np


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--adjoint", action="store_true")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args(argv)

    import torch

    from fvgen.nested import nested_pair
    from paper_1408_5715_amd import fvgpu, learned

    p = learned.load_params()
    c, f, idx, w = nested_pair(1024, 2)
    U0 = learned.Restriction(idx, w, f.n, 1, torch)(
        torch.tensor(learned.flows(f, 10.0 / 1024, [5000])[0], device="cuda"))
    dt = 2 * learned.mesh_dt(f, 0.8)
    s = fvgpu.Solver(c.nbr, c.nrm, c.area)
    s.renumber()
    s.set_correction(p)
    s.upload_state(U0)
    s.step(200, dt)  # warm-up: clocks settle
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    s.step(args.steps, dt)
    ev[1].record()
    torch.cuda.synchronize()
    print(f"corrected step, {c.n} cells: {ev[0].elapsed_time(ev[1]) * 1e3 / args.steps:.1f} us "
          f"per step (HIP events)", flush=True)
    s.close()
    if args.probe_copy:
        # known traffic: 256 MiB read and 256 MiB written per launch
        src = torch.ones(32 * 2**20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
    if args.adjoint:
        cc = nested_pair(128, 1)[0]
        B = 32
        bs = learned.batch_solver(cc, B, torch)
        bs.set_correction(p)
        U = torch.tensor(np.concatenate(learned.flows(cc, 10.0 / 128, range(1000, 1000 + B))),
                         device="cuda")
        lam = torch.ones_like(U)
        g = torch.zeros(fvgpu.FV_CORRECTION_PARAMS, dtype=torch.float64, device="cuda")
        dtc = learned.mesh_dt(cc, 0.8)
        for _ in range(4):
            fvgpu.fv_step_adjoint_grad(bs.ctx, U, lam, dtc, g)
        torch.cuda.synchronize()
        print(f"corrected adjoint, {bs.n} cells: 4 steps done", flush=True)
        bs.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
