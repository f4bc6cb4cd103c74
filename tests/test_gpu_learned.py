"""The learned flux correction on the GPU (BF16 MFMA MLP, FP32 accumulation,
FP64 flux and update), through the C ABI.

Bars against the CPU reference (oracle/learned_ref.py, pinned by hand-worked
values).  Both round the same features, weights and activations to
bfloat16 and sum in float32, in different orders.  Where both round every
activation alike, the corrected steps differ only by the float32 summation
order and float64 arithmetic: about 1e-7 of a row's output, about 1e-6 of
the largest correction effect after a few steps (SUM_ORDER below).  A
pre-activation whose two float32 values straddle a bfloat16 rounding
boundary (a flip) changes its activation by one bfloat16 unit, at most 2^-7
of itself, and so moves its row's output by 2^-7 of that activation's
contribution, about 2^-7 / sqrt(64) ~ 1e-3 of a typical row output.  Flips
are rare: the float32 order difference (~1e-7 relative) against the
bfloat16 spacing (2^-8) makes them of order 1e-5 per activation, so in the
small cases (a few hundred thousand activations per step) none is expected
in the cells with the largest corrections and the bars are 100x the
summation-order level; on larger meshes flips do occur, and the worst cell
is bounded by two flips of a contribution as large as the largest
correction (TWO_FLIPS = 2 * 2^-8), while 99 % of the cells stay at the
summation-order level.  Everything the correction cannot touch stays exact:
conservation to round-off, and zero parameters give the plain step."""

import numpy as np
import pytest
import torch as _torch

import oracle
import paper_1408_5715_amd as fv
from gpu_helpers import TOL, log, rel_err, vortex_case
from oracle import learned_ref, torch_ref

pytestmark = pytest.mark.gpu

SUM_ORDER = 1e-6  # float32 summation order and float64 arithmetic, largest effect's scale
TWO_FLIPS = 2 * 2.0**-8  # two bfloat16 flips of a contribution as large as the largest effect


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
    # 512 cells x 6 rows x 128 activations per step: no flip expected where
    # it matters; later steps feed the difference back through the features
    assert err <= (100 if steps == 1 else 1000) * SUM_ORDER


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
    # 51,200 cells x 3 steps: flips occur
    assert err <= TWO_FLIPS


def test_interleaved_offsets_bitwise(torch):
    """A mesh beyond the Infinity Cache (1200 x 1200 quads, 2,880,000
    cells) keeps its 16-bit offsets interleaved with dt/V once renumbered,
    and the corrected step reads them at a 16-byte stride.  The corrected
    step gives the same bits in any cell order, so the renumbered run and
    the uploaded-order run (32-bit ids) must agree bit for bit."""
    from gpu_helpers import bumps_case

    log("corrected step, interleaved offsets, 1200")
    m, U0, dt = bumps_case(1200)
    assert m.n * 96 > 256 << 20
    p = learned_ref.random_params(4)
    a = run(m, U0, dt, 2, p, fv.FV_ORDER_CM)
    b = run(m, U0, dt, 2, p, fv.FV_ORDER_IDENTITY)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    plain = run(m, U0, dt, 2, None, fv.FV_ORDER_CM)
    assert not np.array_equal(a, plain)


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
        assert err <= 100 * SUM_ORDER


def test_corrected_step_full_size_every_cell(torch):
    """512 x 512 quads (524,288 cells), the trained parameters, 2 corrected
    steps in Cuthill-McKee order, compared with the CPU reference cell by
    cell: the correction's effect on each cell against the largest effect."""
    from paper_1408_5715_amd import learned

    m, U0, dt = vortex_case(512)
    p = learned.load_params()
    log("corrected step: 512 x 512 quads, 2 steps, trained parameters")
    got = run(m, U0, dt, 2, p, fv.FV_ORDER_CM)
    plain = run(m, U0, dt, 2, None, fv.FV_ORDER_CM)
    M = torch_ref.Mesh(m.nbr, m.nrm, m.area)
    Ur, Up = _torch.from_numpy(U0), _torch.from_numpy(U0)
    with _torch.no_grad():
        for _ in range(2):
            Ur = learned_ref.corrected_step(M, Ur, dt, p)
            Up = torch_ref.step(M, Up, dt)
    d_ref = (Ur - Up).numpy()
    d_gpu = got - plain
    scale = np.max(np.abs(d_ref), axis=0)
    cell_err = np.abs(d_gpu - d_ref) / scale
    err = float(cell_err.max())
    per_cell = cell_err.max(1)
    q = {k: float(np.quantile(per_cell, k)) for k in (0.5, 0.9, 0.99, 0.999)}
    log(f"512x512: correction effect vs reference, worst cell {err:.2e} of the largest effect "
        f"per component {scale}; quantiles {q}; cells beyond 1e-6: {int(np.sum(per_cell > 1e-6))}, "
        f"beyond 1e-5: {int(np.sum(per_cell > 1e-5))}, beyond 1e-4: {int(np.sum(per_cell > 1e-4))}")
    assert np.all(rel_err(plain, oracle.step(m.nbr, m.nrm, m.area, U0, dt, 2)) <= TOL)
    # most cells see no flip: summation-order agreement; the few that do
    # (and their neighbours after the second step) stay within two flips
    assert q[0.5] <= SUM_ORDER
    assert q[0.99] <= 100 * SUM_ORDER
    assert np.mean(per_cell > 100 * SUM_ORDER) <= 0.01
    assert err <= TWO_FLIPS
