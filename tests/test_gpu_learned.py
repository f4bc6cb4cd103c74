"""The learned flux correction on the GPU (BF16 MFMA MLP, FP32 accumulation,
FP64 flux and update), through the C ABI.

Bar against the CPU reference (oracle/learned_ref.py): the reference rounds
the same features, weights and activations to bfloat16 but sums in a
different order, so a pre-activation can land on the other side of a
bfloat16 rounding boundary; each such flip changes an activation by at most
2^-8 of itself.  The effect of the correction on the state (corrected minus
plain) must therefore agree to 2 % of its size, while everything the
correction cannot touch stays exact: conservation to round-off, and zero
parameters give the plain step."""

import numpy as np
import pytest
import torch as _torch

import oracle
import paper_1408_5715_amd as fv
from gpu_helpers import TOL, log, rel_err, vortex_case
from oracle import learned_ref, torch_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    assert _torch.cuda.is_available(), "GPU tests need a GPU"
    return _torch


def run(m, U0, dt, steps, params, order=fv.FV_ORDER_IDENTITY, grid=0, nrm=None):
    s = fv.Solver(m.nbr, m.nrm if nrm is None else nrm, m.area)
    try:
        s.upload_state(U0)
        s.renumber(order)
        s.set_correction(params)
        s.set_launch(256, grid, False)
        s.step(steps, dt)
        return s.download()
    finally:
        s.close()


def test_zero_parameters_is_the_plain_step(torch):
    m, U0, dt = vortex_case(24)
    zero = np.zeros(fv.FV_CORRECTION_PARAMS, np.float32)
    got = run(m, U0, dt, 50, zero, fv.FV_ORDER_CM)
    ref = oracle.step(m.nbr, m.nrm, m.area, U0, dt, 50)
    assert np.all(rel_err(got, ref) <= TOL)
    plain = run(m, U0, dt, 50, None, fv.FV_ORDER_CM)
    assert np.all(rel_err(got, plain) <= 1e-14)


@pytest.mark.parametrize("order", [fv.FV_ORDER_IDENTITY, fv.FV_ORDER_CM])
def test_correction_conserves(torch, order):
    m, U0, dt = vortex_case(40)
    p = learned_ref.random_params(1)
    U = run(m, U0, dt, 100, p, order)
    w = m.area[:, None]
    mom = np.sum(m.area * np.hypot(U0[:, 1], U0[:, 2]))
    scale = np.array([np.sum(w[:, 0] * U0[:, 0]), mom, mom, np.sum(w[:, 0] * U0[:, 3])])
    drift = np.abs(np.sum(w * U, 0) - np.sum(w * U0, 0)) / scale
    log(f"conservation drift with the correction: {drift}")
    assert np.all(drift <= 1e-13)
    plain = run(m, U0, dt, 100, None, order)
    assert np.max(np.abs(U - plain)) > 1e-6  # the correction does act


@pytest.mark.parametrize("steps", [1, 5])
def test_matches_cpu_reference(torch, steps):
    m, U0, dt = vortex_case(16)
    p = learned_ref.random_params(2)
    got = run(m, U0, dt, steps, p, fv.FV_ORDER_CM)
    plain = run(m, U0, dt, steps, None, fv.FV_ORDER_CM)
    M = torch_ref.Mesh(m.nbr, m.nrm, m.area)
    U = _torch.from_numpy(U0)
    Ur, Up = U, U
    for _ in range(steps):
        Ur = learned_ref.corrected_step(M, Ur, dt, p)
        Up = torch_ref.step(M, Up, dt)
    d_gpu, d_ref = got - plain, (Ur - Up).numpy()
    err = np.max(np.abs(d_gpu - d_ref)) / np.max(np.abs(d_ref))
    log(f"correction effect after {steps} step(s): GPU vs CPU reference relative {err:.2e}, "
        f"effect size {np.max(np.abs(d_ref)):.2e}")
    assert err <= 2e-2


def test_launch_shapes_and_batches_bitwise(torch):
    """Persistent grids of any size give the same bits (each MLP row depends
    only on its own inputs, whatever its position in an MFMA tile), and a
    mesh inside a batch evolves as it does alone."""
    m, U0, dt = vortex_case(30)
    p = learned_ref.random_params(3)
    ref = run(m, U0, dt, 20, p, fv.FV_ORDER_CM)
    for grid in (1, 5, 8, 64, 100000):
        assert np.array_equal(run(m, U0, dt, 20, p, fv.FV_ORDER_CM, grid=grid), ref), grid
    a, Ua, dta = vortex_case(12, perm_seed=3)
    n = a.n + m.n
    s = fv.Solver(np.concatenate([a.nbr, m.nbr + a.n]), np.concatenate([a.nrm, m.nrm]),
                  np.concatenate([a.area, m.area]), mesh_begin=[0, a.n, n])
    try:
        s.upload_state(np.concatenate([Ua, U0]))
        s.renumber(fv.FV_ORDER_CM)
        s.set_correction(p)
        s.step(20, np.array([dta, dt]))
        got = s.download()
    finally:
        s.close()
    assert np.array_equal(got[a.n:], ref)
    assert np.array_equal(got[:a.n], run(a, Ua, dta, 20, p, fv.FV_ORDER_CM))


@pytest.mark.parametrize("closed", [True, False])
def test_layout_variants(torch, closed):
    """The four geometry layouts of the corrected step (16-bit offsets or
    32-bit ids, derived or stored third normal) give the same bits for runs
    that differ only in the cell order, and match the CPU reference."""
    from test_gpu_step import open_normals

    N = 160  # a random order has neighbour offsets beyond 16 bits, CM's do not
    m, U0, dt = vortex_case(N)
    nrm = m.nrm if closed else open_normals(m)
    p = learned_ref.random_params(4)
    a = run(m, U0, dt, 3, p, fv.FV_ORDER_IDENTITY, nrm=nrm)
    b = run(m, U0, dt, 3, p, fv.FV_ORDER_CM, nrm=nrm)
    assert np.array_equal(a, b)
    plain = run(m, U0, dt, 3, None, fv.FV_ORDER_CM, nrm=nrm)
    M = torch_ref.Mesh(m.nbr, nrm, m.area)
    Ur, Up = _torch.from_numpy(U0), _torch.from_numpy(U0)
    for _ in range(3):
        Ur = learned_ref.corrected_step(M, Ur, dt, p)
        Up = torch_ref.step(M, Up, dt)
    d_ref = (Ur - Up).numpy()
    err = np.max(np.abs((b - plain) - d_ref)) / np.max(np.abs(d_ref))
    log(f"layout closed={closed}: correction effect vs reference {err:.2e}")
    assert err <= 2e-2


def test_graph_replays_and_tiny_meshes(torch):
    """A captured graph of corrected steps replays to the eager bits (several
    replays, eager work in between), and the smallest meshes (2 x 2 quads,
    where a cell meets the same neighbour across two faces) match the CPU
    reference."""
    m, U0, dt = vortex_case(20)
    p = learned_ref.random_params(6)
    eager = run(m, U0, dt, 12, p, fv.FV_ORDER_CM)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.renumber(fv.FV_ORDER_CM)
        s.set_correction(p)
        s.set_launch(256, 0, True)
        for rep in range(3):
            s.upload_state(U0)
            s.step(12, dt)
            got = s.download()
            assert np.array_equal(got, eager), rep
            s.set_launch(256, 0, False)
            s.step(1, dt)  # eager work between replays
            s.set_launch(256, 0, True)
    finally:
        s.close()
    for N in (2, 3):
        m, U0, dt = vortex_case(N)
        got = run(m, U0, dt, 4, p, fv.FV_ORDER_CM)
        plain = run(m, U0, dt, 4, None, fv.FV_ORDER_CM)
        M = torch_ref.Mesh(m.nbr, m.nrm, m.area)
        Ur, Up = _torch.from_numpy(U0), _torch.from_numpy(U0)
        for _ in range(4):
            Ur = learned_ref.corrected_step(M, Ur, dt, p)
            Up = torch_ref.step(M, Up, dt)
        d_ref = (Ur - Up).numpy()
        err = np.max(np.abs((got - plain) - d_ref)) / np.max(np.abs(d_ref))
        log(f"N={N}: correction effect vs reference {err:.2e}")
        assert err <= 2e-2
