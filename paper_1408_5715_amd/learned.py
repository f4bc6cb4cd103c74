"""Training and evaluation of the learned face-flux correction.

Training (coarse N x N mesh, targets from the plain solver on the r-times
refined mesh):
  1. a batch of seeded flows is advanced on the fine mesh by the plain step
     (one batched launch per step for all flows) and restricted to the
     coarse mesh after every r fine steps (fv_restrict: area-weighted means
     over the nested fine cells), giving target trajectories;
  2. each iteration rolls the corrected coarse solver out for `window` steps
     from a restricted state (all flows at once, one batched mesh), scores
     the area-weighted squared density error against the targets at every
     step, and takes the gradient through the hand-written adjoint
     (autograd.rollout, checkpoints every `checkpoint` steps);
  3. Adam updates the float32 parameters.
Evaluation compares the plain and the corrected coarse solvers with the
plain fine solver, restricted, over long rollouts.

Every step, adjoint step and restriction runs in the HIP library; torch holds
device memory, forms the loss and runs the optimiser on the 5252 parameters.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import fvgpu
from .fvgpu import FV_CORRECTION_PARAMS, Solver

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_PARAMS = os.path.join(HERE, "correction_params.npy")
N_IN, N_HID, N_OUT = 12, 64, 4


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised hidden layers, zero output layer (the plain solver)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_IN, N_HID)) * np.sqrt(2.0 / N_IN)
    b1 = np.zeros(N_HID)
    W2 = rng.standard_normal((N_HID, N_HID)) * np.sqrt(2.0 / N_HID)
    b2 = np.zeros(N_HID)
    W3 = np.zeros((N_HID, N_OUT))
    b3 = np.zeros(N_OUT)
    p = np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)
    assert p.size == FV_CORRECTION_PARAMS
    return p


def load_params(path: str = DEFAULT_PARAMS) -> np.ndarray:
    p = np.load(path, allow_pickle=False)
    if p.shape != (FV_CORRECTION_PARAMS,) or p.dtype != np.float32:
        raise ValueError(f"{path}: expected float32 [{FV_CORRECTION_PARAMS}]")
    return p


def _log(msg: str) -> None:
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


def batch_solver(mesh, copies: int, torch):
    """One Solver holding `copies` independent copies of a mesh."""
    n = mesh.n
    nbr = np.concatenate([mesh.nbr + b * n for b in range(copies)]).astype(np.int32)
    nrm = np.concatenate([mesh.nrm] * copies)
    area = np.concatenate([mesh.area] * copies)
    begin = np.arange(copies + 1, dtype=np.int64) * n
    return Solver(nbr, nrm, area, mesh_begin=begin)


def flows(mesh, h: float, seeds):
    from fvgen import ic

    return [ic.to_conserved(ic.flow_primitive(mesh.centroid, h, int(s))) for s in seeds]


# Bound on |v| + c for the flows of fvgen.ic.flow_primitive (stream <= 0.71,
# vortex velocity <= 0.64 each, c <= 1.2 where the bumps raise p).
SIGNAL_SPEED = 3.0


def mesh_dt(mesh, cfl: float) -> float:
    """dt = cfl min_i V_i / (P_i s) with the fixed signal-speed bound s: the
    same for every flow, so dt / V (a feature of the correction) only
    depends on the mesh, and meshes of any resolution see the same values."""
    return float(cfl * np.min(mesh.area / (mesh.perimeter * SIGNAL_SPEED)))


class Restriction:
    """Device-side restriction of a batch of fine states to the coarse mesh."""

    def __init__(self, idx: np.ndarray, w: np.ndarray, n_fine: int, copies: int, torch):
        nc = idx.shape[0]
        off = (np.arange(copies, dtype=np.int64) * n_fine)[:, None, None]
        self.idx = torch.tensor((idx[None].astype(np.int64) + off).reshape(copies * nc, -1)
                                .astype(np.int32), device="cuda")
        self.w = torch.tensor(np.tile(w, (copies, 1)), device="cuda")
        self.torch = torch

    def __call__(self, U_fine, out=None):
        if out is None:
            out = self.torch.empty((self.idx.shape[0], 4), dtype=self.torch.float64,
                                   device="cuda")
        fvgpu.fv_restrict(U_fine, self.idx, self.w, out)
        return out


def make_targets(N: int, r: int, seeds, n_coarse_steps: int, cfl: float, torch):
    """Restricted fine trajectories: tensor [n_coarse_steps + 1, B n_c, 4],
    the coarse mesh and the coarse time step (r fine steps)."""
    from fvgen.nested import nested_pair

    coarse, fine, idx, w = nested_pair(N, r)
    h = 10.0 / N
    dt_f = mesh_dt(fine, cfl)
    B = len(seeds)
    fs = batch_solver(fine, B, torch)
    try:
        fs.upload_state(np.concatenate(flows(fine, h, seeds)))
        R = Restriction(idx, w, fine.n, B, torch)
        T = torch.empty((n_coarse_steps + 1, B * coarse.n, 4), dtype=torch.float64, device="cuda")
        U = fs.download_device()
        R(U, T[0])
        for t in range(1, n_coarse_steps + 1):
            fs.step(r, np.full(B, dt_f))
            fs.download_device(U)
            R(U, T[t])
        torch.cuda.synchronize()
    finally:
        fs.close()
    return T, coarse, r * dt_f


def density_error(torch, U, T, area):
    """Area-weighted squared density error summed over cells, per leading index."""
    return ((U[..., 0] - T[..., 0]) ** 2 * area).sum(-1)


def train(N=128, r=4, n_flows=32, window=16, checkpoint=4, horizon=256, iters=4000, lr=5e-4,
          cfl=0.8, seed=0, params0=None, log_every=100, clip=1.0, max_lead=160):
    """Train the correction; returns (params, history).

    max_lead > 0: each window starts from the corrected solver's own state
    after up to max_lead steps (run without gradient from a restricted
    state; the bound grows linearly over the first half of training), so the
    correction also learns from the states it produces itself, which keeps
    long rollouts stable; the gradient still flows through `window` steps."""
    import torch

    from .autograd import rollout

    seeds = list(range(1000, 1000 + n_flows))
    t0 = time.time()
    T, coarse, dt_c = make_targets(N, r, seeds, horizon, cfl, torch)
    _log(f"targets: {n_flows} flows on {N * r}x{N * r} quads restricted to {N}x{N}, "
         f"{horizon} coarse steps (dt {dt_c:.3e}) in {time.time() - t0:.1f}s")
    cs = batch_solver(coarse, n_flows, torch)
    area = torch.tensor(np.tile(coarse.area, n_flows), device="cuda")
    P = torch.tensor(init_params(seed) if params0 is None else params0, requires_grad=True)
    opt = torch.optim.Adam([P], lr=lr)
    warm = max(1, iters // 20)
    sched = torch.optim.lr_scheduler.LambdaLR(
        opt, lambda k: min(1.0, (k + 1) / warm) * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * k / iters))))
    rng = np.random.default_rng(seed)

    # plain-solver error of every window start, the scale of the loss
    plain = []
    with torch.no_grad():
        for s0 in range(horizon - window + 1):
            out = rollout(T[s0], cs, window, dt_c, checkpoint, None, 1)
            plain.append(float(density_error(torch, out, T[s0 + 1:s0 + window + 1], area).sum()))
    cs.set_correction(None)
    history = []
    for it in range(iters):
        lead = 0
        if max_lead:
            lead = int(rng.integers(0, 1 + int(max_lead * min(1.0, 2.0 * it / iters))))
        s0 = int(rng.integers(0, horizon - window - lead + 1))
        U0 = T[s0]
        if lead:
            with torch.no_grad():
                U0 = rollout(T[s0], cs, lead, dt_c, checkpoint, P, 0)
        s0 += lead
        out = rollout(U0, cs, window, dt_c, checkpoint, P, 1)
        err = density_error(torch, out, T[s0 + 1:s0 + window + 1], area).sum()
        loss = err / plain[s0]
        opt.zero_grad()
        loss.backward()
        torch.nn.utils.clip_grad_norm_([P], clip)
        opt.step()
        sched.step()
        history.append(float(loss.detach()))
        if it % log_every == 0 or it == iters - 1:
            _log(f"iter {it}: window at {s0}, error / plain error {history[-1]:.4f} "
                 f"({time.time() - t0:.0f}s)")
        if not np.isfinite(history[-1]):
            raise RuntimeError("training diverged")
    cs.close()
    return P.detach().numpy().copy(), history


def compare(params, N: int, r: int, seeds, steps: int, cfl: float = 0.8,
            timing_steps: int = 0):
    """Plain coarse, corrected coarse and plain fine solvers from the same
    restricted initial state; returns area-weighted L2 density errors of the
    coarse solvers against the restricted fine solution (per flow, at the
    end), and step timings."""
    import torch

    from fvgen.nested import nested_pair

    coarse, fine, idx, w = nested_pair(N, r)
    h = 10.0 / N
    dt_f = mesh_dt(fine, cfl)
    dt_c = r * dt_f
    R = Restriction(idx, w, fine.n, 1, torch)
    res = {"coarse_cells": coarse.n, "fine_cells": fine.n, "steps": steps, "dt_coarse": dt_c,
           "flows": []}
    area = torch.tensor(coarse.area, device="cuda")
    A = float(coarse.area.sum())
    fs = Solver(fine.nbr, fine.nrm, fine.area)
    cs = Solver(coarse.nbr, coarse.nrm, coarse.area)
    fs.renumber()  # Cuthill-McKee: the step then runs with its compact layout
    cs.renumber()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    try:
        for s in seeds:
            U0f = flows(fine, h, [s])[0]
            fs.upload_state(U0f)
            Uf = fs.download_device()
            U0c = R(Uf).clone()
            rec = {"seed": int(s), "t_end": steps * dt_c}
            fs.step(r * steps, dt_f)
            Tf = R(fs.download_device())
            outs = {}
            for name, p in (("plain", None), ("corrected", params)):
                cs.set_correction(p)
                cs.upload_state(U0c)
                cs.step(steps, dt_c)
                Uc = cs.download_device()
                e = float(torch.sqrt(density_error(torch, Uc, Tf, area) / A))
                outs[name] = e
            rec["l2_rho_plain_vs_fine"] = outs["plain"]
            rec["l2_rho_corrected_vs_fine"] = outs["corrected"]
            rec["ratio"] = outs["corrected"] / outs["plain"]
            res["flows"].append(rec)
            _log(f"seed {s}: L2 density error vs fine: plain {outs['plain']:.3e}, corrected "
                 f"{outs['corrected']:.3e} (ratio {rec['ratio']:.3f})")
        if timing_steps:
            st = torch.cuda.current_stream()
            for name, solver, p, n_steps, dt in (("fine_plain", fs, None, r * timing_steps, dt_f),
                                                 ("coarse_plain", cs, None, timing_steps, dt_c),
                                                 ("coarse_corrected", cs, params, timing_steps,
                                                  dt_c)):
                if solver is cs:
                    cs.set_correction(p)
                    cs.upload_state(U0c)
                solver.step(5, dt)
                a, b = ev(), ev()
                torch.cuda.synchronize()
                a.record(st)
                solver.step(n_steps, dt)
                b.record(st)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                n = solver.n
                res[name] = {"us_per_step": ms * 1e3 / n_steps,
                             "cell_updates_per_s": n * n_steps / (ms * 1e-3)}
    finally:
        fs.close()
        cs.close()
    return res


def compare_levels(params, N: int, seeds, horizons, cfl: float = 0.8) -> dict:
    """Plain and corrected N x N solvers, the plain 2N x 2N solver and a plain
    4N x 4N reference, all from the reference's initial state restricted to
    each mesh; L2 density errors against the reference restricted to N x N
    after each number of coarse steps in `horizons` (2 and 4 substeps per
    coarse step on the finer meshes), and of both coarse solvers against the
    restricted 2N solution.  Answers whether the corrected coarse solver
    reaches the 2N solver's accuracy."""
    import torch

    from fvgen.nested import nested_pair

    c, ref, idx4, w4 = nested_pair(N, 4)
    _log(f"meshes {N}x{N} and {4 * N}x{4 * N} built")
    mid, _, idx2f, w2f = nested_pair(2 * N, 2)
    _, _, idx2, w2 = nested_pair(N, 2)
    _log(f"mesh {2 * N}x{2 * N} built")
    h = 10.0 / N
    dt_r = mesh_dt(ref, cfl)
    R4 = Restriction(idx4, w4, ref.n, 1, torch)  # reference -> coarse
    Rrm = Restriction(idx2f, w2f, ref.n, 1, torch)  # reference -> 2N
    R2 = Restriction(idx2, w2, mid.n, 1, torch)  # 2N -> coarse
    del idx4, w4, idx2f, w2f, idx2, w2
    area = torch.tensor(c.area, device="cuda")
    A = float(c.area.sum())
    horizons = sorted(int(k) for k in horizons)
    out = {"N": N, "horizons": horizons, "dt_coarse": 4 * dt_r, "flows": []}
    rs = Solver(ref.nbr, ref.nrm, ref.area)
    ms = Solver(mid.nbr, mid.nrm, mid.area)
    cs = Solver(c.nbr, c.nrm, c.area)
    for s in (rs, ms, cs):
        s.renumber()

    def err(U, T):
        return float(torch.sqrt(density_error(torch, U, T, area) / A))

    def run(solver, U0, sub, dt, restrict, p=None):
        """restricted (coarse-mesh) states after each horizon"""
        if solver is cs:
            cs.set_correction(p)
        solver.upload_state(U0)
        done, states = 0, []
        for k in horizons:
            solver.step(sub * (k - done), dt)
            done = k
            U = solver.download_device()
            states.append(restrict(U).clone() if restrict else U)
        return states

    try:
        for seed in seeds:
            rs.upload_state(flows(ref, h, [seed])[0])
            _log(f"seed {seed}: reference state uploaded")
            U0r = rs.download_device()
            U0m, U0c = Rrm(U0r).clone(), R4(U0r).clone()
            T = run(rs, U0r, 4, dt_r, R4)
            Em = run(ms, U0m, 2, 2 * dt_r, R2)
            Ep = run(cs, U0c, 1, 4 * dt_r, None)
            Ec = run(cs, U0c, 1, 4 * dt_r, None, params)
            for q, k in enumerate(horizons):
                rec = {"seed": int(seed), "steps": k, "coarse_plain": err(Ep[q], T[q]),
                       "coarse_corrected": err(Ec[q], T[q]), "fine_plain": err(Em[q], T[q]),
                       # against the restricted 2N x 2N plain solution instead
                       "coarse_plain_vs_fine": err(Ep[q], Em[q]),
                       "coarse_corrected_vs_fine": err(Ec[q], Em[q])}
                out["flows"].append(rec)
                _log(f"N={N} seed {seed} {k} steps, L2 density error vs the {4 * N}x{4 * N} "
                     f"reference: coarse plain {rec['coarse_plain']:.3e}, coarse corrected "
                     f"{rec['coarse_corrected']:.3e}, {2 * N}x{2 * N} plain "
                     f"{rec['fine_plain']:.3e}")
    finally:
        for s in (rs, ms, cs):
            s.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--N", type=int, default=128)
    t.add_argument("--r", type=int, default=4)
    t.add_argument("--flows", type=int, default=32)
    t.add_argument("--window", type=int, default=16)
    t.add_argument("--checkpoint", type=int, default=4)
    t.add_argument("--horizon", type=int, default=256)
    t.add_argument("--iters", type=int, default=4000)
    t.add_argument("--lr", type=float, default=5e-4)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--max-lead", type=int, default=160)
    t.add_argument("--out", default=DEFAULT_PARAMS)
    t.add_argument("--history", default="")
    e = sub.add_parser("compare")
    e.add_argument("--N", type=int, default=128)
    e.add_argument("--r", type=int, default=4)
    e.add_argument("--steps", type=int, default=64)
    e.add_argument("--seeds", default="2000,2001")
    e.add_argument("--params", default=DEFAULT_PARAMS)
    e.add_argument("--timing-steps", type=int, default=0)
    args = ap.parse_args(argv)
    if args.cmd == "train":
        p, hist = train(args.N, args.r, args.flows, args.window, args.checkpoint, args.horizon,
                        args.iters, args.lr, seed=args.seed, max_lead=args.max_lead)
        np.save(args.out, p.astype(np.float32), allow_pickle=False)
        if args.history:
            with open(args.history, "w") as f:
                json.dump(hist, f)
        _log(f"saved {args.out}")
    else:
        p = load_params(args.params)
        res = compare(p, args.N, args.r, [int(s) for s in args.seeds.split(",")], args.steps,
                      timing_steps=args.timing_steps)
        print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
