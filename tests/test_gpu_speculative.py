"""fv_renumber without perm_out does not wait for the root search's
confirming sweep: the labels assume the search stays at its first
candidate, the sweep runs on the context's second stream beside the steps,
and the next call that needs it checks it (and relabels exactly if the
search would have moved).  Every result must equal the synchronous path's:
the states bit for bit, the working order and the pass counts element by
element, on a mesh whose search stays, on ladders whose search moves, and on
a batch holding both."""

import numpy as np
import pytest

import oracle
import paper_1408_5715_amd as fv
from gpu_helpers import bumps_case, george_liu_passes, ladder_graph, log, vortex_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def shuffled_ladder(length, seed):
    nbr, nrm, area = ladder_graph(length)
    p0 = np.random.default_rng(seed).permutation(nbr.shape[0])
    inv0 = np.empty_like(p0)
    inv0[p0] = np.arange(p0.size)
    return inv0[nbr[p0]].astype(np.int32), nrm[p0], area[p0]


def smooth_state(n, seed):
    rng = np.random.default_rng(seed)
    U = np.tile(np.array([1.0, 0.1, 0.05, 2.5]), (n, 1))
    return U * (1.0 + 0.01 * rng.standard_normal(U.shape))


def run(torch, nbr, nrm, area, U0, dt, steps, speculative, mesh_begin=None):
    s = fv.Solver(nbr, nrm, area, mesh_begin=mesh_begin)
    try:
        dU = torch.tensor(U0, device="cuda")
        if speculative:
            fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)  # no perm_out: does not wait
        else:
            s.renumber(fv.FV_ORDER_CM)
        fv.fv_upload_state_device(s.ctx, dU)
        s.step(steps, dt)
        out = s.download_device().cpu().numpy()
        passes = s.renumber_passes()  # checks a pending sweep
        order = s.working_order()
        return out, passes, order
    finally:
        s.close()


def test_search_that_stays(torch):
    m, U0, dt = bumps_case(256)
    a = run(torch, m.nbr, m.nrm, m.area, U0, dt, 30, True)
    b = run(torch, m.nbr, m.nrm, m.area, U0, dt, 30, False)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1]) and int(a[1][0]) == 2
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[2], oracle.cm_order(m.nbr))


@pytest.mark.parametrize("length,seed", [(40, 1), (301, 7)])
def test_search_that_moves(torch, length, seed):
    """The speculation fails: the check relabels, and order and passes equal
    the synchronous search's; the steps taken in the provisional order give
    the same bits."""
    nbr, nrm, area = shuffled_ladder(length, seed)
    U0 = smooth_state(nbr.shape[0], seed)
    dt = 1e-3
    a = run(torch, nbr, nrm, area, U0, dt, 12, True)
    b = run(torch, nbr, nrm, area, U0, dt, 12, False)
    log(f"ladder {length}: passes {int(a[1][0])} (George-Liu {george_liu_passes(nbr)})")
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], oracle.cm_order(nbr))
    assert np.array_equal(a[2], b[2])


def test_batch_with_moving_and_staying_searches(torch):
    meshes = [shuffled_ladder(40, 1)]
    m, _, _ = vortex_case(9, perm_seed=4)
    meshes.append((m.nbr, m.nrm, m.area))
    meshes.append(shuffled_ladder(301, 7))
    begin = np.concatenate([[0], np.cumsum([x[0].shape[0] for x in meshes])]).astype(np.int64)
    nbr = np.concatenate([x[0] + b for x, b in zip(meshes, begin)]).astype(np.int32)
    nrm = np.concatenate([x[1] for x in meshes])
    area = np.concatenate([x[2] for x in meshes])
    U0 = smooth_state(int(begin[-1]), 3)
    dts = np.full(len(meshes), 1e-3)
    a = run(torch, nbr, nrm, area, U0, dts, 8, True, mesh_begin=begin)
    b = run(torch, nbr, nrm, area, U0, dts, 8, False, mesh_begin=begin)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    for k, x in enumerate(meshes):
        lo, hi = begin[k], begin[k + 1]
        assert np.array_equal(a[2][lo:hi] - lo, oracle.cm_order(x[0])), k


def test_pending_sweep_and_every_entry_point(torch):
    """Calls that use the scratch memory or replace the mesh while a sweep is
    pending wait for it: a host state upload, a host download, an adjoint
    step, a new upload of the mesh, a second renumbering, and destroying the
    context."""
    m, U0, dt = bumps_case(128)
    ref = run(torch, m.nbr, m.nrm, m.area, U0, dt, 10, False)[0]
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        s.upload_state(U0)  # host upload: stages through the scratch memory
        s.step(10, dt)
        assert np.array_equal(s.download(), ref)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        dU = torch.tensor(U0, device="cuda")
        lam = torch.ones_like(dU)
        fv.fv_step_adjoint(s.ctx, dU, lam, dt)
        assert torch.isfinite(lam).all()
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        fv.fv_upload_mesh(s.ctx, m.nbr, m.nrm, m.area)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        s.upload_state(U0)
        s.step(10, dt)
        assert np.array_equal(s.download(), ref)
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
    finally:
        s.close()  # destroys the context while a sweep may be pending
