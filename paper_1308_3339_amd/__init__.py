"""MI355X (gfx950) FMM-preconditioned Krylov solver for the 5-point Poisson
matrix, after Ibeid, Yokota, Pestana, Keyes (arXiv:1308.3339).

The compute lives in ``libfmmprec.so`` (hand-written HIP, C ABI declared in
``include/fmmprec.h``).  This package only marshals arguments: torch tensors
supply device memory and the current HIP stream.  Importing works without a
GPU; every call needs the built library and a GPU, and raises otherwise.
"""
from ._binding import (  # noqa: F401
    FMM_ERR_ALLOC, FMM_ERR_ARG, FMM_ERR_DEVICE, FMM_ERR_NUMERIC, FMM_ERR_UNSUPPORTED,
    FMM_FP32, FMM_FP64, FMM_SPLIT_BF16, FMM_SPLIT_FP16, FMM_GRID, STAGES, FMM_NOT_CONVERGED, FMM_OK, FMM_POINTS, FmmError, Plan, exported_symbols,
    fmm_apply, fmm_destroy, fmm_last_error, fmm_precond_apply, fmm_precond_stages, fmm_profile, fmm_profile_read, fmm_setup,
    fmm_stencil_apply, fmm_version, library_path, load_library, precond_gmres_solve,
    precond_gmres_solve_adjoint, fmm_bumps_eval, fmm_bumps_grad, fmm_bumps_grad_noalloc, fmm_stencil_var_apply,
    precond_gmres_solve_var, precond_gmres_solve_batch, fmm_tune, fmm_tune_m2l, fmm_set_m2l_split, fmm_get_m2l_split, FMM_BATCH_GRAPHS, FMM_BATCH_SEPARATE, precond_gmres_solve_multi, fmm_points_order, points_levels,
)
