"""Seeded synthetic inputs for the differentiable Gaussian rasterizer.

This package only draws random numbers and arranges them into the parameter
and camera layouts that both the CPU oracle and the HIP path consume.  It
holds none of the rasterizer's arithmetic and imports neither side.
"""
from .generators import (  # noqa: F401
    Camera,
    Scene,
    CONFIGS,
    RIG_LAYOUT,
    make_config,
    make_insert_inputs,
    make_target,
    config_names,
)
