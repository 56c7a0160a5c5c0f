"""Direct Fourier transform of polygonal areas and closed triangulated volumes on MI355X.

The transform F(Q) = integral of exp(iQ.r) over the region is evaluated by the
divergence theorem as sums over polygon edges and mesh faces (Maranville,
"An implementation of an efficient direct Fourier transform of polygonal
areas and volumes"), in hand-written HIP kernels for gfx950 behind the C ABI
declared in include/pft.h. This package is the thin Python binding.
"""
from .api import (  # noqa: F401
    forward_2d, forward_3d, forward_3d_noalloc, forward_3d_poly, backward_3d, batch_forward, batch_backward, orientation_average,
    forward_3d_regions, backward_3d_regions, intensity_loss_3d, strip_order, batch_strip_order, q_order, validate_mesh, check_mesh, fp32c_q_limit,
    profile_enable, profile_reset, profile_read, release_workspace, version, tuning_info,
)
from .autograd import (  # noqa: F401
    IntensityLossFunction, PftFunction, PftRegionsFunction, ft3d, ft3d_regions, fused_intensity_loss, intensity_loss,
)

__version__ = "0.1.0"
