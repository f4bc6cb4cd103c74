"""MI355X (gfx950) explicit finite-volume Euler step on unstructured triangles.

The computation lives in libfvgpu.so (HIP kernels behind the C ABI of
include/fvgpu.h); this package is its thin Python binding.
"""

from .fvgpu import (  # noqa: F401
    EXPORTS,
    FV_EHIP,
    FV_EINVAL,
    FV_EMESH,
    FV_ENOMEM,
    FV_ESTATE,
    FV_OK,
    FV_CORRECTION_PARAMS,
    FV_MAX_CELLS,
    FV_STATIC_MAX_CELLS,
    FV_ORDER_CM,
    FV_ORDER_IDENTITY,
    FVError,
    Solver,
    fv_arena_bytes,
    fv_bytes_per_update,
    fv_check_state,
    fv_create,
    fv_destroy,
    fv_download_state,
    fv_download_state_device,
    fv_last_error,
    fv_renumber,
    fv_renumber_passes,
    fv_set_correction,
    fv_set_launch,
    fv_step_adjoint,
    fv_step_batch,
    fv_step_static,
    fv_upload_batch,
    fv_step,
    fv_upload_mesh,
    fv_upload_state,
    fv_upload_state_device,
    fv_working_order,
    lib,
)
