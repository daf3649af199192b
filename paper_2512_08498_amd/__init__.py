"""MI355X-native differentiable Gaussian rasterizer (forward, adjoint, L1
loss and fused Adam) behind the C ABI of include/gsr.h.

The HIP library ``libgsr.so`` must be built (``python -m
paper_2512_08498_amd.build``); importing the binding raises otherwise.
"""
from .frequency import Frequency  # noqa: F401
from .rasterizer import (  # noqa: F401
    DEFAULT_LR,
    PARAM_NAMES,
    FusedAdam,
    RasterizeFn,
    Rasterizer,
    camera_rows,
    device_copy,
    rasterize,
)
