"""Batched meshes, launch shapes and graph replay on the GPU, through the C ABI.

A batch is several independent periodic meshes stepped together, each with
its own time step; every mesh must evolve exactly as it does alone (bitwise)
and agree with the oracle to the 1e-12 bar."""

import numpy as np
import pytest

import oracle
import paper_1408_5715_amd as fv
from fvgen import ic
from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation
from gpu_helpers import TOL, george_liu_passes, ladder_graph, log, rel_err, vortex_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def make_batch(sizes, seed=0):
    """Meshes of the given quads-per-side, random cell order each, alternating
    vortex and bump states; returns concatenated arrays, offsets, U0, dt."""
    rng = np.random.default_rng(seed)
    parts, Us, dts = [], [], []
    for k, N in enumerate(sizes):
        m = permute_mesh(periodic_mesh(N, seed=100 + k), random_permutation(2 * N * N, 200 + k))
        if k % 2 == 0:
            P = ic.vortex_primitive(m.centroid, center=tuple(rng.uniform(2, 8, 2)))
        else:
            P = ic.bumps_primitive(m.centroid, seed=300 + k)
        parts.append(m)
        Us.append(ic.to_conserved(P))
        dts.append(ic.cfl_dt(P, m.area, m.perimeter))
    begin = np.concatenate([[0], np.cumsum([m.n for m in parts])]).astype(np.int64)
    nbr = np.concatenate([m.nbr + b for m, b in zip(parts, begin)]).astype(np.int32)
    nrm = np.concatenate([m.nrm for m in parts])
    area = np.concatenate([m.area for m in parts])
    return parts, begin, nbr, nrm, area, np.concatenate(Us), np.array(dts), Us


def run_single(m, U0, dt, steps, order):
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        s.renumber(order)
        s.step(steps, dt)
        return s.download()
    finally:
        s.close()


@pytest.mark.parametrize("order", [fv.FV_ORDER_IDENTITY, fv.FV_ORDER_CM])
def test_batch_equals_single_meshes(torch, order):
    sizes = [5, 9, 13, 20, 31, 48]
    parts, begin, nbr, nrm, area, U0, dts, Us = make_batch(sizes)
    log(f"batch of {len(sizes)}: {begin[-1]} cells, order {order}")
    s = fv.Solver(nbr, nrm, area, mesh_begin=begin)
    try:
        s.upload_state(U0)
        perm = s.renumber(order)
        s.step(60, dts)
        got = s.download()
        passes = s.renumber_passes() if order == fv.FV_ORDER_CM else None
    finally:
        s.close()
    for k, m in enumerate(parts):
        lo, hi = begin[k], begin[k + 1]
        alone = run_single(m, Us[k], dts[k], 60, order)
        assert np.array_equal(got[lo:hi], alone), f"mesh {k}"
        if order == fv.FV_ORDER_CM:
            # the batch renumbering keeps each mesh in its own range, in its own CM order
            assert np.array_equal(perm[lo:hi] - lo, oracle.cm_order(m.nbr))
            assert passes[k] >= 2
    for k in (0, 3):
        m = parts[k]
        ref = oracle.step(m.nbr, m.nrm, m.area, Us[k], dts[k], 60)
        assert np.all(rel_err(got[begin[k]:begin[k + 1]], ref) <= TOL)


def test_batch_renumbering_with_moving_searches(torch):
    """A batch of two shuffled ladders (whose pseudo-peripheral search moves,
    so their confirming pass on the renamed graph sees the eccentricity grow
    and the search continues on the original graph) around a periodic mesh
    (whose search stops after the confirmation): every mesh gets its own
    sequential Cuthill-McKee order, with the pass counts that implies."""
    meshes = []
    for length, seed in ((40, 1), (301, 7)):
        nbr, nrm, area = ladder_graph(length)
        rng = np.random.default_rng(seed)
        p0 = rng.permutation(nbr.shape[0])
        inv0 = np.empty_like(p0)
        inv0[p0] = np.arange(p0.size)
        meshes.append((inv0[nbr[p0]].astype(np.int32), nrm[p0], area[p0]))
    m, _, _ = vortex_case(9, perm_seed=4)
    meshes.insert(1, (m.nbr, m.nrm, m.area))
    begin = np.concatenate([[0], np.cumsum([x[0].shape[0] for x in meshes])]).astype(np.int64)
    nbr = np.concatenate([x[0] + b for x, b in zip(meshes, begin)]).astype(np.int32)
    nrm = np.concatenate([x[1] for x in meshes])
    area = np.concatenate([x[2] for x in meshes])
    log(f"batch with moving searches: {begin[-1]} cells")
    s = fv.Solver(nbr, nrm, area, mesh_begin=begin)
    try:
        perm = s.renumber(fv.FV_ORDER_CM)
        passes = s.renumber_passes()
    finally:
        s.close()
    for k, x in enumerate(meshes):
        lo, hi = begin[k], begin[k + 1]
        assert np.array_equal(perm[lo:hi] - lo, oracle.cm_order(x[0])), f"mesh {k}"
        gl = george_liu_passes(x[0])
        # a search that moves counts its confirming pass once more
        assert passes[k] == (gl + 1 if gl > 2 else gl), (k, passes[k], gl)


@pytest.mark.parametrize("block", [128, 256, 512])
def test_launch_shapes_bitwise(torch, block):
    """Block size, persistent grid (including fewer workgroups than XCDs) and
    graph capture change nothing in the result."""
    m, U0, dt = vortex_case(40)
    ref = run_single(m, U0, dt, 50, fv.FV_ORDER_CM)
    for grid in (0, 3, 8, 77, 10_000):
        for graph in (False, True):
            s = fv.Solver(m.nbr, m.nrm, m.area)
            try:
                s.upload_state(U0)
                s.renumber(fv.FV_ORDER_CM)
                s.set_launch(block, grid, graph)
                s.step(50, dt)
                got = s.download()
            finally:
                s.close()
            assert np.array_equal(got, ref), (block, grid, graph)


def test_graph_replays_match_eager(torch):
    """One captured graph replayed several times, with eager work and host
    synchronisation in between; every replay matches the eager result."""
    m, U0, dt = vortex_case(32)
    s = fv.Solver(m.nbr, m.nrm, m.area)
    e = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.upload_state(U0)
        e.upload_state(U0)
        s.renumber(fv.FV_ORDER_CM)
        s.set_launch(256, 0, True)
        for rep in range(4):
            s.step(20, dt)  # same step count and parity -> the cached graph
            e.step(20, dt)
            junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work
            torch.cuda.synchronize()
            assert np.array_equal(s.download(), e.download()), f"replay {rep}"
            del junk
        s.step(7, dt)  # odd count: a new graph, then the parity flips
        e.step(7, dt)
        s.step(7, dt)
        e.step(7, dt)
        assert np.array_equal(s.download(), e.download())
    finally:
        s.close()
        e.close()


def test_batch_per_mesh_dt_changes(torch):
    """Changing the per-mesh time steps between calls re-derives dt / V."""
    sizes = [6, 11]
    parts, begin, nbr, nrm, area, U0, dts, Us = make_batch(sizes, seed=3)
    s = fv.Solver(nbr, nrm, area, mesh_begin=begin)
    try:
        s.upload_state(U0)
        s.step(10, dts)
        s.step(10, dts * 0.5)
        got = s.download()
    finally:
        s.close()
    for k, m in enumerate(parts):
        a = oracle.step(m.nbr, m.nrm, m.area, Us[k], dts[k], 10)
        b = oracle.step(m.nbr, m.nrm, m.area, a, dts[k] * 0.5, 10)
        assert np.all(rel_err(got[begin[k]:begin[k + 1]], b) <= TOL)


@pytest.mark.slow
def test_c3_full_batch(torch, tmp_path):
    """The 64-mesh batch at full size (about 12M cells), renumbered per mesh on
    the GPU, 500 steps in the autotuned launch shape: the smallest mesh
    matches the oracle, a mid-size mesh matches its own single-mesh run
    bitwise, and every mesh conserves mass, momentum and energy.  The batch
    is beyond the Infinity Cache, so it runs the streaming step with its
    offsets interleaved with per-mesh dt/V; the single-mesh runs do not."""
    from fvgen.batch import batch_workload, concat
    from paper_1408_5715_amd import autotune

    log("c3 generate")
    parts, begin, sizes, Us, dts = batch_workload()
    nbr, nrm, area = concat(parts)
    U0 = np.concatenate(Us)
    log(f"c3 gpu {begin[-1]} cells")
    s = fv.Solver(nbr, nrm, area, mesh_begin=begin)
    try:
        s.renumber(fv.FV_ORDER_CM)
        s.upload_state(U0)
        autotune.tune(s, dts, steps=4, cache_path=str(tmp_path / "tune.json"))
        s.upload_state(U0)
        s.step(500, dts)
        got = s.download()
        s.check_state()
    finally:
        s.close()
    k_small = int(np.argmin(sizes))
    m = parts[k_small]
    log(f"c3 oracle on mesh {k_small} ({m.n} cells)")
    ref = oracle.step(m.nbr, m.nrm, m.area, Us[k_small], dts[k_small], 500)
    assert np.all(rel_err(got[begin[k_small]:begin[k_small + 1]], ref) <= TOL)
    k_mid = int(np.argsort(sizes)[len(sizes) // 2])
    alone = run_single(parts[k_mid], Us[k_mid], dts[k_mid], 500, fv.FV_ORDER_CM)
    assert np.array_equal(got[begin[k_mid]:begin[k_mid + 1]], alone)
    for k, mk in enumerate(parts):
        seg = got[begin[k]:begin[k + 1]]
        t0 = np.sum(mk.area[:, None] * Us[k], axis=0)
        t1 = np.sum(mk.area[:, None] * seg, axis=0)
        mom = np.sum(mk.area * np.hypot(Us[k][:, 1], Us[k][:, 2]))
        scale = np.array([np.sum(mk.area * Us[k][:, 0]), mom, mom, np.sum(mk.area * Us[k][:, 3])])
        assert np.all(np.abs(t1 - t0) / scale <= 1e-13), (k, (t1 - t0) / scale)
