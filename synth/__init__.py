"""Seeded synthetic inputs for the MMGKS-OF operators and solver.

This package only draws random numbers and paints phantoms.  It holds none of
the method's arithmetic (no projector, no warp, no derivative, no solver step):
both the FP64 oracle and the HIP path receive the arrays it returns as inputs.
"""
from .workloads import (  # noqa: F401
    Sequence,
    Workload,
    angle_schedule,
    angles_shifted,
    cfg_disk32,
    cfg_krylov210,
    cfg_ellipse128,
    cfg_blur_ragged,
    cfg_autograd256,
    cfg_large1024,
    bins_for,
    noisy,
    random_field,
    smooth_flow,
    smooth_flow_coarse,
    nudge_off_kinks,
    GOLDEN_ANGLE_180,
)
