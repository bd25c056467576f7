"""Seeded synthetic inputs for the shooting workloads.

This package is shared by the tests, the benchmark and the smoke check. It holds
input recipes only (phantoms, random smooth warps, lesions, initial momenta);
smoothing and warping here go through SciPy library routines, and nothing of the
registration method's own arithmetic lives in it.
"""
from .phantoms import (  # noqa: F401
    Pair,
    Workload,
    SIZES_2D,
    SHAPES_3D,
    LAMBDA,
    P0_KINDS,
    gradient_noise,
    phantom,
    smooth_warp,
    warp_image,
    lesion_mask,
    make_p0,
    disk_pair,
    phantom_pair,
    ripple_case,
    workload,
    workload_pair,
    c5_shape_classes,
    small_pair,
    large_step,
    LARGE_STEP_T,
    LARGE_STEP_SCALE,
)
