"""ctypes binding of libfvgpu.so (C ABI declared in include/fvgpu.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions keep the C names; a failing status raises FVError with
the library's message.  PyTorch only supplies device memory (the arena) and
the stream.  There is no fallback: without the built library, loading fails.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfvgpu.so")

FV_OK = 0
FV_EINVAL = -1
FV_EMESH = -2
FV_ESTATE = -3
FV_EHIP = -4
FV_ENOMEM = -5
FV_ORDER_IDENTITY = 0
FV_ORDER_CM = 1
FV_CORRECTION_PARAMS = 5252
FV_MAX_CELLS = 268431360  # largest mesh a context accepts (device offsets are 32-bit)
FV_STATIC_MAX_CELLS = 1048576  # largest mesh fv_step_static takes (its static scratch array)

# every symbol include/fvgpu.h declares
EXPORTS = (
    "fv_arena_bytes", "fv_create", "fv_upload_mesh", "fv_upload_batch", "fv_upload_state",
    "fv_upload_state_device", "fv_renumber", "fv_step", "fv_step_batch", "fv_step_adjoint",
    "fv_step_adjoint_grad", "fv_set_correction", "fv_restrict", "fv_set_launch",
    "fv_renumber_passes", "fv_download_state", "fv_download_state_device", "fv_bytes_per_update",
    "fv_check_state", "fv_destroy", "fv_last_error", "fv_step_static", "fv_working_order",
)


class FVError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fvgpu status {status}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_1408_5715_amd.build` "
                "(the library has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_size_t)
        L.fv_arena_bytes.argtypes = [i64]
        L.fv_arena_bytes.restype = sz
        L.fv_create.argtypes = [i64, dbl, vp, sz, vp, ctypes.POINTER(vp)]
        L.fv_upload_mesh.argtypes = [vp, vp, vp, vp]
        L.fv_upload_batch.argtypes = [vp, i32, vp, vp, vp, vp]
        L.fv_step_batch.argtypes = [vp, i32, vp]
        L.fv_set_launch.argtypes = [vp, i32, i32, i32]
        L.fv_step_adjoint.argtypes = [vp, vp, vp, dbl]
        L.fv_step_adjoint_grad.argtypes = [vp, vp, vp, dbl, vp]
        L.fv_restrict.argtypes = [vp, i64, vp, vp, i64, i32, vp, vp]
        L.fv_step_static.argtypes = [i64, vp, vp, vp, vp, i32, dbl, dbl, vp]
        L.fv_set_correction.argtypes = [vp, vp, i32]
        L.fv_renumber_passes.argtypes = [vp, vp]
        L.fv_upload_state.argtypes = [vp, vp]
        L.fv_upload_state_device.argtypes = [vp, vp]
        L.fv_renumber.argtypes = [vp, i32, vp]
        L.fv_working_order.argtypes = [vp, vp]
        L.fv_step.argtypes = [vp, i32, dbl]
        L.fv_download_state.argtypes = [vp, vp]
        L.fv_download_state_device.argtypes = [vp, vp]
        L.fv_bytes_per_update.argtypes = [vp]
        L.fv_bytes_per_update.restype = i64
        L.fv_check_state.argtypes = [vp]
        L.fv_destroy.argtypes = [vp]
        L.fv_last_error.argtypes = []
        L.fv_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("fv_arena_bytes", "fv_last_error", "fv_bytes_per_update"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(status: int) -> int:
    if status < 0:
        raise FVError(status, fv_last_error())
    return status


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


# --- one wrapper per C entry point ------------------------------------------

def fv_arena_bytes(n_cells: int) -> int:
    return int(lib().fv_arena_bytes(int(n_cells)))


def fv_create(n_cells: int, gamma: float, d_arena, arena_bytes: int, hip_stream) -> int:
    out = ctypes.c_void_p()
    _check(lib().fv_create(int(n_cells), float(gamma), _ptr(d_arena), int(arena_bytes),
                           hip_stream, ctypes.byref(out)))
    return out.value


def fv_upload_mesh(ctx: int, nbr: np.ndarray, nrm: np.ndarray, area: np.ndarray) -> None:
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float64)
    _check(lib().fv_upload_mesh(ctx, _ptr(nbr), _ptr(nrm), _ptr(area)))


def fv_upload_batch(ctx: int, mesh_begin, nbr: np.ndarray, nrm: np.ndarray,
                    area: np.ndarray) -> None:
    mb = np.ascontiguousarray(mesh_begin, dtype=np.int64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float64)
    _check(lib().fv_upload_batch(ctx, int(mb.size - 1), _ptr(mb), _ptr(nbr), _ptr(nrm), _ptr(area)))


def fv_step_batch(ctx: int, n_steps: int, dt) -> None:
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    _check(lib().fv_step_batch(ctx, int(n_steps), _ptr(dt)))


def fv_step_adjoint(ctx: int, d_U, d_lambda, dt: float) -> None:
    _check(lib().fv_step_adjoint(ctx, _ptr(d_U), _ptr(d_lambda), float(dt)))


def fv_step_adjoint_grad(ctx: int, d_U, d_lambda, dt: float, d_grad) -> None:
    """d_grad: float64 device tensor [FV_CORRECTION_PARAMS], accumulated."""
    _check(lib().fv_step_adjoint_grad(ctx, _ptr(d_U), _ptr(d_lambda), float(dt),
                                      None if d_grad is None else _ptr(d_grad)))


def fv_restrict(d_src, d_idx, d_w, d_out, stream=None) -> None:
    """d_out[i] = sum_m d_w[i, m] d_src[d_idx[i, m]] (device tensors: src
    float64 [n_src, 4], idx int32 [n, k], w float64 [n, k], out float64 [n, 4])."""
    n, k = d_idx.shape
    _check(lib().fv_restrict(_ptr(d_src), int(d_src.shape[0]), _ptr(d_idx), _ptr(d_w), int(n),
                             int(k), _ptr(d_out), None if stream is None else stream.cuda_stream))


def fv_step_static(d_nbr, d_nrm, d_area, d_U, n_steps: int, dt: float, gamma: float = 1.4,
                   stream=None) -> None:
    """fv_step without a context or arena (no allocation): device tensors
    nbr int32 [3, n], nrm float64 [6, n], area float64 [n], U float64 [n, 4]
    (advanced in place), scratch in the library's static device array."""
    n = int(d_U.shape[0])
    _check(lib().fv_step_static(n, _ptr(d_nbr), _ptr(d_nrm), _ptr(d_area), _ptr(d_U),
                                int(n_steps), float(dt), float(gamma),
                                None if stream is None else stream.cuda_stream))


def fv_set_correction(ctx: int, params) -> None:
    """params: float32 [FV_CORRECTION_PARAMS], or None for the plain step."""
    if params is None:
        _check(lib().fv_set_correction(ctx, None, 0))
        return
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().fv_set_correction(ctx, _ptr(p), int(p.size)))


def fv_set_launch(ctx: int, block: int = 256, grid: int = 0, use_graph: bool = False) -> None:
    _check(lib().fv_set_launch(ctx, int(block), int(grid), int(bool(use_graph))))


def fv_renumber_passes(ctx: int, n_meshes: int) -> np.ndarray:
    out = np.empty(n_meshes, dtype=np.int32)
    _check(lib().fv_renumber_passes(ctx, _ptr(out)))
    return out


def fv_upload_state(ctx: int, U: np.ndarray) -> None:
    U = np.ascontiguousarray(U, dtype=np.float64)
    _check(lib().fv_upload_state(ctx, _ptr(U)))


def fv_upload_state_device(ctx: int, d_U) -> None:
    _check(lib().fv_upload_state_device(ctx, _ptr(d_U)))


def fv_renumber(ctx: int, method: int, perm_out: np.ndarray | None = None) -> None:
    """Without perm_out, a Cuthill-McKee renumbering does not wait for the
    root search's confirming sweep (see include/fvgpu.h)."""
    _check(lib().fv_renumber(ctx, int(method), _ptr(perm_out)))


def fv_working_order(ctx: int, n: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _check(lib().fv_working_order(ctx, _ptr(perm)))
    return perm


def fv_step(ctx: int, n_steps: int, dt: float) -> None:
    _check(lib().fv_step(ctx, int(n_steps), float(dt)))


def fv_download_state(ctx: int, U: np.ndarray) -> None:
    assert U.dtype == np.float64 and U.flags.c_contiguous
    _check(lib().fv_download_state(ctx, _ptr(U)))


def fv_download_state_device(ctx: int, d_U) -> None:
    _check(lib().fv_download_state_device(ctx, _ptr(d_U)))


def fv_bytes_per_update(ctx: int) -> int:
    return int(lib().fv_bytes_per_update(ctx))


def fv_check_state(ctx: int) -> None:
    _check(lib().fv_check_state(ctx))


def fv_destroy(ctx: int) -> None:
    _check(lib().fv_destroy(ctx))


def fv_last_error() -> str:
    return lib().fv_last_error().decode(errors="replace")


# --- convenience object -------------------------------------------------------

class Solver:
    """One mesh on one GPU: arena from torch, work on torch's current stream."""

    def __init__(self, nbr, nrm, area, gamma: float = 1.4, device="cuda:0", stream=None,
                 mesh_begin=None):
        """mesh_begin (optional): offsets of the independent meshes of a batch."""
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.n = int(np.asarray(nbr).shape[0])
        self.nbytes = fv_arena_bytes(self.n)
        if self.nbytes == 0:
            raise FVError(FV_EINVAL, f"bad cell count {self.n}")
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = fv_create(self.n, gamma, self.arena, self.nbytes, self.stream.cuda_stream)
        if mesh_begin is None:
            self.n_meshes = 1
            fv_upload_mesh(self.ctx, nbr, nrm, area)
        else:
            self.n_meshes = len(mesh_begin) - 1
            fv_upload_batch(self.ctx, mesh_begin, nbr, nrm, area)

    def upload_state(self, U) -> None:
        if isinstance(U, np.ndarray):
            fv_upload_state(self.ctx, U)
        else:
            fv_upload_state_device(self.ctx, U)

    def renumber(self, method: int = FV_ORDER_CM) -> np.ndarray:
        perm = np.empty(self.n, dtype=np.int32)
        fv_renumber(self.ctx, method, perm)
        return perm

    def step(self, n_steps: int, dt) -> None:
        """dt: one value, or one per mesh of a batch."""
        if np.ndim(dt) == 0:
            fv_step(self.ctx, n_steps, float(dt))
        else:
            fv_step_batch(self.ctx, n_steps, dt)

    def set_correction(self, params) -> None:
        fv_set_correction(self.ctx, params)

    def set_launch(self, block: int = 256, grid: int = 0, use_graph: bool = False) -> None:
        fv_set_launch(self.ctx, block, grid, use_graph)

    def working_order(self) -> np.ndarray:
        return fv_working_order(self.ctx, self.n)

    def renumber_passes(self) -> np.ndarray:
        return fv_renumber_passes(self.ctx, self.n_meshes)

    def download(self) -> np.ndarray:
        U = np.empty((self.n, 4), dtype=np.float64)
        fv_download_state(self.ctx, U)
        return U

    def download_device(self, out=None):
        if out is None:
            out = self.torch.empty((self.n, 4), dtype=self.torch.float64, device=self.device)
        fv_download_state_device(self.ctx, out)
        return out

    def check_state(self) -> None:
        fv_check_state(self.ctx)

    def bytes_per_update(self) -> int:
        return fv_bytes_per_update(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            fv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
