"""The C ABI on a machine without a GPU: the library loads, exports every
symbol include/fvgpu.h declares, and rejects bad input on the host before any
HIP call (so these calls never touch a device)."""

import ctypes
import os
import re
import threading

import numpy as np
import pytest

import paper_1408_5715_amd as fv
from fvgen.mesh import shuffled_periodic_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE_ARENA = 1 << 20  # never dereferenced: validation fails first


def header_functions():
    text = open(os.path.join(ROOT, "include", "fvgpu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fv_\w+)\s*\(", text)))


def test_exports_match_header():
    declared = header_functions()
    assert declared == sorted(fv.EXPORTS)
    L = fv.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_arena_bytes():
    assert fv.fv_arena_bytes(0) == 0
    assert fv.fv_arena_bytes(-5) == 0
    assert fv.fv_arena_bytes(1 << 31) == 0
    # device offsets such as 6 ld + i are 32-bit: the bound keeps 8 ld < 2^31
    assert fv.FV_MAX_CELLS == (1 << 28) - 4096
    assert fv.fv_arena_bytes(fv.FV_MAX_CELLS) > 0
    assert fv.fv_arena_bytes(fv.FV_MAX_CELLS + 1) == 0
    assert fv.fv_arena_bytes((1 << 31) - 4096) == 0
    b = fv.fv_arena_bytes(8192)
    # fixed parts: the per-mesh tables of a batch (up to 65536 meshes, 2.4 MB)
    # and the correction's weights and per-workgroup gradients (512 x 5252 floats)
    fixed = (3 << 20) + 512 * 5252 * 4 + (64 << 10)
    assert 240 * 8192 <= b <= 300 * 8192 + fixed
    assert fv.fv_arena_bytes(8193) >= b
    big = fv.fv_arena_bytes(1 << 21)
    assert 250 * (1 << 21) <= big <= 300 * (1 << 21) + fixed


def make_ctx(n):
    return fv.fv_create(n, 1.4, FAKE_ARENA, fv.fv_arena_bytes(n), None)


def test_create_rejects_bad_arguments():
    n = 128
    nb = fv.fv_arena_bytes(n)
    cases = [
        (0, 1.4, FAKE_ARENA, nb),
        (n, 1.0, FAKE_ARENA, nb),
        (n, float("nan"), FAKE_ARENA, nb),
        (n, 1.4, 0, nb),
        (n, 1.4, FAKE_ARENA + 8, nb),
        (n, 1.4, FAKE_ARENA, nb - 1),
        (fv.FV_MAX_CELLS + 1, 1.4, FAKE_ARENA, 1 << 40),
        (1 << 30, 1.4, FAKE_ARENA, 1 << 40),
    ]
    for args in cases:
        with pytest.raises(fv.FVError) as e:
            fv.fv_create(*args, None)
        assert e.value.status == fv.FV_EINVAL, args
    ctx = make_ctx(n)
    fv.fv_destroy(ctx)


@pytest.fixture
def mesh():
    return shuffled_periodic_mesh(8)


def expect(status, fn, *args):
    with pytest.raises(fv.FVError) as e:
        fn(*args)
    assert e.value.status == status
    return str(e.value)


def test_mesh_validation(mesh):
    ctx = make_ctx(mesh.n)
    try:
        nbr = mesh.nbr.copy()
        nbr[5, 1] = mesh.n
        assert "out of range" in expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, nbr, mesh.nrm, mesh.area)
        nbr = mesh.nbr.copy()
        nbr[5, 1] = 5
        assert "own neighbour" in expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, nbr, mesh.nrm, mesh.area)
        nbr = mesh.nbr.copy()
        nbr[5, 1] = mesh.nbr[6, 0]
        expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, nbr, mesh.nrm, mesh.area)
        nrm = mesh.nrm.copy()
        nrm[7, 2, 0] = np.nextafter(nrm[7, 2, 0], np.inf)
        assert "negated" in expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, mesh.nbr, nrm, mesh.area)
        nrm = mesh.nrm.copy()
        nrm[3, 0] = np.nan
        expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, mesh.nbr, nrm, mesh.area)
        area = mesh.area.copy()
        area[9] = 0.0
        assert "area" in expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, mesh.nbr, mesh.nrm, area)
        area[9] = np.inf
        expect(fv.FV_EMESH, fv.fv_upload_mesh, ctx, mesh.nbr, mesh.nrm, area)
    finally:
        fv.fv_destroy(ctx)


def test_calls_before_upload_and_bad_step_arguments(mesh):
    ctx = make_ctx(mesh.n)
    try:
        U = np.tile([1.0, 0.0, 0.0, 2.5], (mesh.n, 1))
        expect(fv.FV_ESTATE, fv.fv_upload_state, ctx, U)
        expect(fv.FV_ESTATE, fv.fv_step, ctx, 1, 1e-3)
        expect(fv.FV_EINVAL, fv.fv_step, ctx, -1, 1e-3)
        expect(fv.FV_EINVAL, fv.fv_step, ctx, 1, 0.0)
        expect(fv.FV_EINVAL, fv.fv_step, ctx, 1, float("nan"))
        expect(fv.FV_EINVAL, fv.fv_step, ctx, 1, float("inf"))
        expect(fv.FV_EINVAL, fv.fv_renumber, ctx, 7)
        expect(fv.FV_ESTATE, fv.fv_renumber, ctx, fv.FV_ORDER_CM)
        expect(fv.FV_ESTATE, fv.fv_download_state, ctx, np.empty((mesh.n, 4)))
        expect(fv.FV_ESTATE, fv.fv_check_state, ctx)
        expect(fv.FV_EINVAL, fv.fv_upload_state_device, ctx, FAKE_ARENA + 8)
    finally:
        fv.fv_destroy(ctx)


def test_null_context():
    L = fv.lib()
    assert L.fv_step(None, 1, ctypes.c_double(1e-3)) == fv.FV_EINVAL
    assert L.fv_destroy(None) == fv.FV_EINVAL
    assert "null" in fv.fv_last_error()


def test_last_error_is_per_thread():
    L = fv.lib()
    assert L.fv_destroy(None) == fv.FV_EINVAL
    seen = {}

    def other():
        seen["msg"] = fv.fv_last_error()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == ""
    assert fv.fv_last_error() != ""


def test_batch_validation():
    from fvgen.mesh import periodic_mesh

    a, b = periodic_mesh(4), periodic_mesh(5)
    n = a.n + b.n
    nbr = np.concatenate([a.nbr, b.nbr + a.n])
    nrm = np.concatenate([a.nrm, b.nrm])
    area = np.concatenate([a.area, b.area])
    ctx = make_ctx(n)
    try:
        for bad in ([0, a.n], [1, a.n, n], [0, a.n, n - 1], [0, a.n, a.n, n], [0, n + 1]):
            expect(fv.FV_EINVAL, fv.fv_upload_batch, ctx, bad, nbr, nrm, area)
        # one mesh split across two segments: faces cross the boundary
        assert "another segment" in expect(fv.FV_EMESH, fv.fv_upload_batch, ctx,
                                          [0, a.n // 2, n], nbr, nrm, area)
        expect(fv.FV_EINVAL, fv.fv_set_launch, ctx, 64, 0, False)
        expect(fv.FV_EINVAL, fv.fv_set_launch, ctx, 256, -1, False)
        assert fv.lib().fv_set_launch(ctx, 256, 0, 2) == fv.FV_EINVAL
        fv.fv_set_launch(ctx, 512, 1024, True)
        expect(fv.FV_ESTATE, fv.fv_step_batch, ctx, 1, np.ones(2))
        assert fv.lib().fv_step_batch(ctx, 1, None) == fv.FV_EINVAL
        expect(fv.FV_ESTATE, fv.fv_renumber_passes, ctx, 2)
    finally:
        fv.fv_destroy(ctx)
