"""Cell orders on the GPU: random, AM1 (the paper's section 4.2 labelling,
computed by the CPU reference) and GPU Cuthill-McKee, on the 1024 x 1024-quad
mesh.  Results must be bitwise identical whatever the order; the step time
and the bandwidth metrics of section 4.1 are printed for each order (the
analog of the paper's Table 1 and of its renumbered-vs-not CPU comparison)."""

import numpy as np
import pytest

import oracle
import paper_1408_5715_amd as fv
from fvgen.mesh import permute_mesh
from gpu_helpers import bumps_case, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def timed_run(torch, m, U0, dt, order, steps=200):
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        s.renumber(order)
        s.step(20, dt)
        out = s.download()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.step(steps, dt)
        b.record(s.stream)
        torch.cuda.synchronize()
        return out, a.elapsed_time(b) * 1e3 / steps, s.bytes_per_update()
    finally:
        s.close()


@pytest.mark.slow
def test_orders_on_c2(torch):
    m, U0, dt = bumps_case(1024)
    lab = lambda p: np.argsort(p).astype(np.int64)  # noqa: E731
    log("orders: AM1 and CM on the CPU")
    p_am1 = oracle.am1_order(m.nbr).astype(np.int64)
    p_cm = oracle.cm_order(m.nbr).astype(np.int64)
    rows = []
    ref, us, bpu = timed_run(torch, m, U0, dt, fv.FV_ORDER_IDENTITY)
    rows.append(("random", oracle.bandwidth(m.nbr, np.arange(m.n)), us, bpu))
    ma = permute_mesh(m, p_am1)
    got, us, bpu = timed_run(torch, ma, U0[p_am1], dt, fv.FV_ORDER_IDENTITY)
    back = np.empty_like(got)
    back[p_am1] = got
    assert np.array_equal(back, ref)
    rows.append(("AM1", oracle.bandwidth(m.nbr, lab(p_am1)), us, bpu))
    got, us, bpu = timed_run(torch, m, U0, dt, fv.FV_ORDER_CM)
    assert np.array_equal(got, ref)
    rows.append(("GPU CM", oracle.bandwidth(m.nbr, lab(p_cm)), us, bpu))
    for name, bw, us, bpu in rows:
        log(f"order {name:7s} B {bw['B']:8d} C_BW {bw['C_BW']:8d} S_BW {bw['S_BW']:8d} "
            f"step {us:8.2f} us  layout {bpu} B/cell")
