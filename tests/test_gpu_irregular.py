"""The path on meshes of irregular topology (random diagonals and edge
flips, fvgen.mesh.irregular_periodic_mesh), where breadth-first levels are
uneven and AM1 and Cuthill-McKee give different orders: GPU Cuthill-McKee
equals the oracle's order element by element, the step matches the oracle at
1e-12 and gives the same bits in every order, and the orders are compared on
the section 4.1 metrics and the step time (the analog of the paper's Table 1
and of its renumbered-vs-random comparison).

When run under `rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum` (profile.sh
orders), the comparison's step launches come in three runs of COMMON +
RUNS[order] launches each, in the order random, AM1, Cuthill-McKee, so the
L2 hit rate of each order can be read off the dispatch sequence."""

import time

import numpy as np
import pytest

import oracle
import paper_1408_5715_amd as fv
from fvgen import ic
from fvgen.mesh import irregular_periodic_mesh, permute_mesh, random_permutation
from gpu_helpers import TOL, log, rel_err

pytestmark = pytest.mark.gpu

COMMON = 20  # steps compared across the orders, before the timed runs
RUNS = {"random": 150, "AM1": 200, "CM": 250}


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def case(N, seed, vortex=True, refine=None):
    m = irregular_periodic_mesh(N, seed=seed, refine=refine)
    m = permute_mesh(m, random_permutation(m.n, seed + 100))
    P = ic.vortex_primitive(m.centroid) if vortex else ic.bumps_primitive(m.centroid, seed=3)
    return m, ic.to_conserved(P), ic.cfl_dt(P, m.area, m.perimeter, 0.4)


@pytest.mark.parametrize("N,seed,steps,refine", [(48, 6, 100, None), (256, 7, 20, None),
                                                 (40, 8, 50, (6.0, 4.0, 2.0, 3))])
def test_irregular_cm_and_step_parity(torch, N, seed, steps, refine):
    m, U0, dt = case(N, seed, refine=refine)
    log(f"irregular {N}x{N} (seed {seed}, refine {refine}, {m.n} cells): GPU Cuthill-McKee and "
        f"{steps} steps vs the oracle")
    ref_perm = oracle.cm_order(m.nbr)
    ref = oracle.step(m.nbr, m.nrm, m.area, U0, dt, steps)
    outs = []
    for order in (fv.FV_ORDER_CM, fv.FV_ORDER_IDENTITY):
        s = fv.Solver(m.nbr, m.nrm, m.area)
        try:
            s.upload_state(U0)
            perm = s.renumber(order)
            if order == fv.FV_ORDER_CM:
                assert np.array_equal(perm, ref_perm)
                log(f"  passes {int(s.renumber_passes()[0])}, layout {s.bytes_per_update()} B/cell")
            s.step(steps, dt)
            outs.append(s.download())
        finally:
            s.close()
    assert np.all(rel_err(outs[0], ref) <= TOL), rel_err(outs[0], ref)
    assert np.array_equal(outs[0], outs[1])


def timed(torch, m, U0, dt, order, steps):
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.renumber(order)
        b.record(s.stream)
        torch.cuda.synchronize()
        renum_ms = a.elapsed_time(b)
        s.step(COMMON, dt)
        out = s.download()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.step(steps, dt)
        b.record(s.stream)
        torch.cuda.synchronize()
        return out, a.elapsed_time(b) * 1e3 / steps, s.bytes_per_update(), renum_ms
    finally:
        s.close()


@pytest.mark.slow
def test_orders_on_irregular_mesh(torch):
    N = 512
    m, U0, dt = case(N, 11, vortex=False)
    lab = lambda p: np.argsort(p).astype(np.int64)  # noqa: E731
    t0 = time.perf_counter()
    p_am1 = oracle.am1_order(m.nbr).astype(np.int64)
    t_am1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    p_cm = oracle.cm_order(m.nbr).astype(np.int64)
    t_cm = time.perf_counter() - t0
    rows = []
    ref, us, bpu, _ = timed(torch, m, U0, dt, fv.FV_ORDER_IDENTITY, RUNS["random"])
    rows.append(("random", oracle.bandwidth(m.nbr, np.arange(m.n, dtype=np.int32)), us, bpu, None))
    ma = permute_mesh(m, p_am1)
    got, us, bpu, _ = timed(torch, ma, U0[p_am1], dt, fv.FV_ORDER_IDENTITY, RUNS["AM1"])
    back = np.empty_like(got)
    back[p_am1] = got
    assert np.array_equal(back, ref)
    rows.append(("AM1", oracle.bandwidth(m.nbr, lab(p_am1).astype(np.int32)), us, bpu,
                 f"CPU {t_am1:.2f} s"))
    got, us, bpu, gms = timed(torch, m, U0, dt, fv.FV_ORDER_CM, RUNS["CM"])
    assert np.array_equal(got, ref)
    rows.append(("CM", oracle.bandwidth(m.nbr, lab(p_cm).astype(np.int32)), us, bpu,
                 f"CPU {t_cm:.2f} s, GPU {gms:.1f} ms"))
    for name, bw, us, bpu, t in rows:
        log(f"irregular {N}x{N} order {name:6s} B {bw['B']:8d} C_BW {bw['C_BW']:8d} "
            f"S_BW {bw['S_BW']:8d} step {us:8.2f} us layout {bpu} B/cell "
            f"{'' if t is None else 'ordering ' + t}")
    assert rows[1][2] < rows[0][2] and rows[2][2] < rows[0][2]
