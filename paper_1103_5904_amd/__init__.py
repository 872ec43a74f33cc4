"""MI355X (gfx950) implementation of TomograPy's hot path: the Siddon
line-of-sight projector P, its exact transpose P^T, and conjugate-gradient
inversion of (P^T P + lambda D^T D) x = P^T y, as HIP kernels behind the C ABI
in include/tomo.h.  This package is the thin Python binding."""
from .tomo import (  # noqa: F401
    NPARAMS, Batch, ConvNet, adam_step, autotune, autotune_clear, class_tuning,
    BP_ATOMIC, BP_AUTO, BP_BINNED, BP_BLOCKED, DeviceGeometry, TomoError, apply_prior, backproject,
    backproject_noalloc, binning_spills, cg_solve, cg_workspace_bytes, get_tuning, set_tuning,
    count_crossings, lib, project, status_string, thomson_backproject, thomson_project, trace_ray, validate,
    view_from_wcs,
)
