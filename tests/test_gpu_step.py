"""GPU parity of the HIP step, renumbering and permutation against the CPU
oracle, through the C ABI.  Bar: per-component relative max error <= 1e-12
(the oracle does not contract FMAs, the GPU does; see gpu_helpers.TOL);
bitwise wherever the arithmetic is the same (re-runs, renumbering, resume)."""

import math

import numpy as np
import pytest

import oracle
import paper_1408_5715_amd as fv
from gpu_helpers import (TOL, bumps_case, conserved_totals, george_liu_passes, ladder_graph, log,
                         rel_err, vortex_case)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def run_gpu(m, U0, dt, steps, order=fv.FV_ORDER_IDENTITY, chunks=None):
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        perm = s.renumber(order) if order != fv.FV_ORDER_IDENTITY else None
        for k in chunks or [steps]:
            s.step(k, dt)
        return s.download(), perm
    finally:
        s.close()


@pytest.mark.parametrize("N", [2, 3, 13, 64])
def test_c1_parity_200_steps(torch, N):
    """The 64 x 64 periodic vortex case (8,192 cells, CFL 0.4, 200 steps) and
    smaller meshes below one workgroup and with a ragged last workgroup."""
    log(f"parity N={N}")
    m, U0, dt = vortex_case(N)
    ref = oracle.step(m.nbr, m.nrm, m.area, U0, dt, 200)
    got, _ = run_gpu(m, U0, dt, 200)
    err = rel_err(got, ref)
    assert np.all(err <= TOL), err


def test_bit_stable_and_order_independent(torch):
    m, U0, dt = vortex_case(64)
    a, _ = run_gpu(m, U0, dt, 200)
    b, _ = run_gpu(m, U0, dt, 200)
    c, perm = run_gpu(m, U0, dt, 200, order=fv.FV_ORDER_CM)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
    assert not np.array_equal(perm, np.arange(m.n))


@pytest.mark.parametrize("N,seed", [(2, 1), (3, 2), (16, 5), (37, 2), (64, 2), (100, 8)])
def test_gpu_cm_equals_oracle_cm(torch, N, seed):
    log(f"cm N={N} seed={seed}")
    m, U0, _ = vortex_case(N, perm_seed=seed)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        perm = s.renumber(fv.FV_ORDER_CM)
    finally:
        s.close()
    assert np.array_equal(perm, oracle.cm_order(m.nbr))


def test_gpu_cm_disconnected_mesh(torch):
    """Two meshes side by side (two components): the labelling restarts on
    the component of the lowest unlabelled id, as in the oracle."""
    a, _, _ = vortex_case(5, perm_seed=3)
    b, _, _ = vortex_case(7, perm_seed=4)
    n = a.n + b.n
    nbr = np.concatenate([a.nbr, b.nbr + a.n])
    nrm = np.concatenate([a.nrm, b.nrm])
    area = np.concatenate([a.area, b.area])
    rng = np.random.default_rng(0)
    perm0 = rng.permutation(n)
    inv0 = np.empty(n, dtype=np.int64)
    inv0[perm0] = np.arange(n)
    nbr = inv0[nbr[perm0]].astype(np.int32)
    nrm, area = nrm[perm0], area[perm0]
    s = fv.Solver(nbr, nrm, area)
    try:
        perm = s.renumber(fv.FV_ORDER_CM)
    finally:
        s.close()
    assert np.array_equal(perm, oracle.cm_order(nbr))


def test_renumber_identity_restores_order(torch):
    m, U0, dt = vortex_case(16)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        s.step(5, dt)
        s.renumber(fv.FV_ORDER_CM)
        s.step(5, dt)
        perm = s.renumber(fv.FV_ORDER_IDENTITY)
        s.step(5, dt)
        got = s.download()
    finally:
        s.close()
    assert np.array_equal(perm, np.arange(m.n))
    ref, _ = run_gpu(m, U0, dt, 15)
    assert np.array_equal(got, ref)


def test_checkpoint_resume_bitwise(torch):
    m, U0, dt = vortex_case(32)
    full, _ = run_gpu(m, U0, dt, 200, order=fv.FV_ORDER_CM)
    half, _ = run_gpu(m, U0, dt, 100, order=fv.FV_ORDER_CM)
    resumed, _ = run_gpu(m, half, dt, 100, order=fv.FV_ORDER_CM)
    assert np.array_equal(full, resumed)
    chunked, _ = run_gpu(m, U0, dt, 200, chunks=[1, 0, 99, 37, 63])
    assert np.array_equal(full, chunked)


def test_zero_steps_roundtrip(torch):
    m, U0, dt = vortex_case(9)
    got, _ = run_gpu(m, U0, dt, 0, order=fv.FV_ORDER_CM)
    assert np.array_equal(got, U0)


def test_every_cell_written(torch):
    """Fill the output buffer with NaN bytes before a step: every cell must be
    overwritten (no thread may skip its cell)."""
    m, U0, dt = vortex_case(37)
    ref = oracle.step(m.nbr, m.nrm, m.area, U0, dt, 1)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        perm = s.renumber(fv.FV_ORDER_CM)
        ld = (m.n + 63) // 64 * 64
        # the arena starts with the two state buffers (32 bytes per cell
        # each); the one holding the state in the working order is the
        # step's input, the other its output
        work = np.ascontiguousarray(U0[perm]).view(np.uint8).reshape(-1)
        first = s.arena[: m.n * 32].cpu().numpy()
        out = 1 if np.array_equal(first, work) else 0
        if out == 0:
            assert np.array_equal(s.arena[ld * 32: ld * 32 + m.n * 32].cpu().numpy(), work)
        s.arena[out * ld * 32: out * ld * 32 + m.n * 32].fill_(0xFF)
        torch.cuda.synchronize()
        s.step(1, dt)
        got = s.download()
    finally:
        s.close()
    assert np.all(np.isfinite(got))
    assert np.all(rel_err(got, ref) <= TOL)


def test_device_resident_state_roundtrip(torch):
    m, U0, dt = vortex_case(20)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        dU = torch.from_numpy(U0).cuda()
        s.upload_state(dU)
        s.renumber(fv.FV_ORDER_CM)
        s.step(10, dt)
        out = s.download_device()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        s.close()
    ref, _ = run_gpu(m, U0, dt, 10)
    assert np.array_equal(got, ref)


def test_state_checks(torch):
    m, U0, dt = vortex_case(16)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        bad = U0.copy()
        bad[3, 0] = -1.0
        with pytest.raises(fv.FVError) as e:
            s.upload_state(bad)
        assert e.value.status == fv.FV_ESTATE
        s.upload_state(U0)
        s.check_state()
        # a step 200 times past the CFL limit loses positivity
        s.step(20, 200 * dt)
        with pytest.raises(fv.FVError) as e:
            s.check_state()
        assert e.value.status == fv.FV_ESTATE
    finally:
        s.close()


@pytest.mark.slow
def test_c2_full_size(torch):
    """The 1024 x 1024-quad mesh (2,097,152 cells) with the bump state: GPU in
    random order and in GPU Cuthill-McKee order against the oracle after 20
    steps (every cell compared), then 1000 steps: the two orders stay bitwise
    equal and mass, momentum and energy are conserved to round-off."""
    log("c2 mesh")
    m, U0, dt = bumps_case(1024)
    log("c2 oracle 20 steps")
    ref = oracle.step(m.nbr, m.nrm, m.area, U0, dt, 20)
    log("c2 gpu")
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        s.step(20, dt)
        a5 = s.download()
        assert np.all(rel_err(a5, ref) <= TOL), rel_err(a5, ref)
        s.upload_state(U0)
        s.step(1000, dt)
        a = s.download()
        perm = s.renumber(fv.FV_ORDER_CM)
        s.upload_state(U0)
        s.step(20, dt)
        b5 = s.download()
        s.upload_state(U0)
        s.step(1000, dt)
        b = s.download()
        s.check_state()
    finally:
        s.close()
    assert np.array_equal(a5, b5)
    assert np.array_equal(a, b)
    log("c2 cm check")
    assert np.array_equal(perm, oracle.cm_order(m.nbr))
    t0 = conserved_totals(m, U0)
    t1 = conserved_totals(m, a)
    # momentum relative to the total |momentum| (the y-momentum total is 0)
    mom = np.sum(m.area * np.hypot(U0[:, 1], U0[:, 2]))
    scale = np.array([np.sum(m.area * U0[:, 0]), mom, mom, np.sum(m.area * U0[:, 3])])
    assert np.all(np.abs(t1 - t0) / scale <= 1e-13), (t1 - t0) / scale


def double_tree_graph(depth: int):
    """A 3-regular graph with very wide BFS levels: two ternary-rooted binary
    trees whose leaves are joined in a ring (leaf i of one tree to leaves i and
    i + 1 of the other).  Faces get placeholder normals that are exactly
    antisymmetric, so the mesh validator accepts it; only the renumbering is
    exercised on it."""
    def tree(offset):
        nodes = [[offset]]
        edges = []
        nid = offset + 1
        for d in range(depth):
            kids = 3 if d == 0 else 2
            level = []
            for p in nodes[-1]:
                for _ in range(kids):
                    edges.append((p, nid))
                    level.append(nid)
                    nid += 1
            nodes.append(level)
        return nodes[-1], edges, nid

    leavesA, eA, nxt = tree(0)
    leavesB, eB, n = tree(nxt)
    edges = eA + eB
    L = len(leavesA)
    for i in range(L):
        edges.append((leavesA[i], leavesB[i]))
        edges.append((leavesA[i], leavesB[(i + 1) % L]))
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    assert all(len(a) == 3 for a in adj)
    nbr = np.array(adj, dtype=np.int32)
    nrm = np.empty((n, 3, 2))
    for u in range(n):
        for f, v in enumerate(adj[u]):
            sgn = 1.0 if u < v else -1.0
            nrm[u, f] = (sgn * 1.0, sgn * 0.5)
    return nbr, nrm, np.ones(n)


def test_gpu_cm_wide_levels(torch):
    """Levels far wider than the LDS tables hold (over 12,000 cells): the
    renumbering falls back to labels in global memory and still matches the
    sequential order exactly."""
    nbr, nrm, area = double_tree_graph(13)
    rng = np.random.default_rng(5)
    p0 = rng.permutation(nbr.shape[0])
    inv0 = np.empty_like(p0)
    inv0[p0] = np.arange(p0.size)
    nbr, nrm, area = inv0[nbr[p0]].astype(np.int32), nrm[p0], area[p0]
    log(f"wide levels: {nbr.shape[0]} cells")
    s = fv.Solver(nbr, nrm, area)
    try:
        perm = s.renumber(fv.FV_ORDER_CM)
    finally:
        s.close()
    assert np.array_equal(perm, oracle.cm_order(nbr))


@pytest.mark.parametrize("length,seed", [(40, 1), (301, 7)])
def test_gpu_cm_search_that_moves(torch, length, seed):
    """The eccentricity grows from the first pick: the GPU search leaves its
    confirmation pass on the renamed graph and continues on the original one,
    and its order equals the sequential order exactly."""
    nbr, nrm, area = ladder_graph(length)
    rng = np.random.default_rng(seed)
    p0 = rng.permutation(nbr.shape[0])
    inv0 = np.empty_like(p0)
    inv0[p0] = np.arange(p0.size)
    nbr, nrm, area = inv0[nbr[p0]].astype(np.int32), nrm[p0], area[p0]
    gl = george_liu_passes(nbr)
    log(f"ladder {length} seed {seed}: {gl} search passes")
    assert gl >= 3
    s = fv.Solver(nbr, nrm, area)
    try:
        perm = s.renumber(fv.FV_ORDER_CM)
        passes = int(s.renumber_passes()[0])
    finally:
        s.close()
    assert np.array_equal(perm, oracle.cm_order(nbr))
    # one extra pass: the confirmation on the renamed graph that saw the growth
    assert passes == gl + 1


def test_fixed_point_normals_only_when_exact(torch):
    """A closed mesh whose faces are longer than 1/2 keeps its normals in
    float64 (112 bytes per update) and still matches the oracle; the
    fixed-point form of a fine snapped mesh decodes to the same bits as the
    float64 one (the corrected step with zero parameters reads the float64
    normals and equals the plain step bitwise, tested with the correction)."""
    m, U0, dt = vortex_case(8)  # h = 1.25
    assert np.abs(m.nrm).max() >= 0.5
    ref = oracle.step(m.nbr, m.nrm, m.area, U0, dt, 50)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        assert s.bytes_per_update() == 32 + 32 + 8 + 8 + 32
        s.step(50, dt)
        got = s.download()
    finally:
        s.close()
    assert np.all(rel_err(got, ref) <= TOL), rel_err(got, ref)
    fine, _, _ = vortex_case(64)
    assert np.any((fine.nrm == 0.0) & np.signbit(fine.nrm))  # -0.0 components occur
    s = fv.Solver(fine.nbr, fine.nrm, fine.area)
    try:
        assert s.bytes_per_update() == 32 + 32 + 8 + 8 + 16
    finally:
        s.close()


def open_normals(m, fraction=0.05, seed=9):
    """Scale the normals of some face pairs by (1 + 2^-20) on both sides:
    antisymmetry stays exact, closure n_2 = -(n_0 + n_1) no longer holds."""
    nrm = m.nrm.copy()
    rng = np.random.default_rng(seed)
    for i in rng.choice(m.n, max(1, int(fraction * m.n)), replace=False):
        f = 0
        j = m.nbr[i, f]
        g = [g for g in range(3) if m.nbr[j, g] == i and np.all(m.nrm[j, g] == -m.nrm[i, f])][0]
        nrm[i, f] *= 1.0 + 2.0**-20
        nrm[j, g] = -nrm[i, f]
    return nrm


@pytest.mark.parametrize("closed", [True, False])
@pytest.mark.parametrize("order", [fv.FV_ORDER_IDENTITY, fv.FV_ORDER_CM])
def test_layout_variants(torch, closed, order):
    """The geometry layouts of the step (16-bit offsets or 32-bit ids;
    normals in fixed point with the third derived, or the third derived, or
    all stored) agree with the oracle."""
    N = 160  # 51,200 cells: a random order has offsets beyond 16 bits, CM's do not
    m, U0, dt = vortex_case(N)
    nrm = m.nrm if closed else open_normals(m)
    log(f"layout closed={closed} order={order}")
    ref = oracle.step(m.nbr, nrm, m.area, U0, dt, 100)
    s = fv.Solver(m.nbr, nrm, m.area)
    try:
        s.upload_state(U0)
        s.renumber(order)
        # the snapped mesh's normals are multiples of 2^-32 well below 1/2
        want = 32 + 32 + 8 + (8 if order == fv.FV_ORDER_CM else 12) + (16 if closed else 48)
        assert s.bytes_per_update() == want
        s.step(100, dt)
        got = s.download()
    finally:
        s.close()
    assert np.all(rel_err(got, ref) <= TOL), rel_err(got, ref)


@pytest.mark.slow
def test_2048_mesh_beyond_the_cache(torch):
    """The 2048 x 2048-quad mesh (8,388,608 cells) that bench.py times beyond
    the Infinity Cache, in the same launch configuration (renumbered on the
    GPU without waiting for the confirming sweep, one workgroup per tile):
    10 steps against the oracle on every cell (the oracle's cell loop on the
    host's cores, which gives its bits), and the layout is the compact one."""
    import os

    log("2048 mesh")
    m, U0, dt = bumps_case(2048)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        fv.fv_renumber(s.ctx, fv.FV_ORDER_CM)
        assert s.bytes_per_update() == 96
        fv.fv_upload_state_device(s.ctx, torch.tensor(U0, device="cuda"))
        s.step(10, dt)
        got = s.download_device().cpu().numpy()
        assert int(s.renumber_passes()[0]) == 2
    finally:
        s.close()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    log(f"2048 oracle 10 steps on {threads} threads")
    ref, _ = oracle.default().step_threads(m.nbr, m.nrm, m.area, U0, dt, 10, threads)
    err = rel_err(got, ref)
    log(f"2048 mesh, 10 steps: {err}")
    assert np.all(err <= TOL), err


@pytest.mark.slow
@pytest.mark.parametrize("layout,bytes_per_update", [("compact", 96), ("float64 normals", 112),
                                                      ("open normals", 128)])
def test_streaming_step_equals_cached_step_bitwise(torch, layout, bytes_per_update):
    """A renumbered mesh whose working set exceeds the 256 MB Infinity Cache
    (1200 x 1200 quads, 2,880,000 cells: 276 MB in the compact layout, 322
    MB with float64 normals, 369 MB with all three normals stored) takes the
    step variant with non-temporal reads of its per-cell arrays and its
    16-bit offsets interleaved with dt/V; on the uploaded (random) order it
    takes the 32-bit index variant without them.  A step gives the same bits
    in any cell order, so the two runs must agree bit for bit, also after a
    change of dt (which rewrites the interleaved dt/V)."""
    log(f"streaming step 1200, {layout}")
    m, U0, dt = bumps_case(1200, snap_bits=40 if layout == "float64 normals" else 32)
    nrm = open_normals(m) if layout == "open normals" else m.nrm
    assert m.n * bytes_per_update > 256 << 20
    a = fv.Solver(m.nbr, nrm, m.area)
    b = fv.Solver(m.nbr, nrm, m.area)
    try:
        a.upload_state(U0)
        a.renumber(fv.FV_ORDER_CM)
        assert a.bytes_per_update() == bytes_per_update
        a.step(5, dt)
        a.step(3, 0.5 * dt)
        got = a.download()
        b.upload_state(U0)
        b.step(5, dt)
        b.step(3, 0.5 * dt)
        ref = b.download()
    finally:
        a.close()
        b.close()
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
