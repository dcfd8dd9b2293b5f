"""MI355X-native DiffCloud hot path (arXiv 2204.03139): area-weighted surface sampling, the
bidirectional / unidirectional Chamfer distance, and the backward pass to mesh vertices, as HIP
kernels for gfx950 behind a C ABI (libdiffcloud.so, declared in include/diffcloud.h).

The Python layer only marshals torch device tensors to that ABI.
"""
from ._lib import (  # noqa: F401
    DC_PREC_FP32, DC_PREC_BF16_REFINE, DC_RED_BIDIR_MEAN, DC_RED_SIM2REAL_SUM, DCError, Context,
    area_cdf, chamfer_bwd, chamfer_fwd, default_context, load, rigid_pose, rigid_pose_bwd,
    sample_surface, sample_surface_bwd, sample_surface_noalloc,
)
from .autograd import DiffCloudChamfer, RigidPose, diffcloud_loss  # noqa: F401
