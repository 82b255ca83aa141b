"""Seeded synthetic test images for the shiftable bilateral filter.

This package only draws random numbers and paints shapes.  It holds none of
the filter's arithmetic, so both the FP64 oracle and the GPU path may use it
to obtain identical inputs.
"""
from .synth import (  # noqa: F401
    CONFIGS,
    config_image,
    batch_images,
    gen_rect_u8,
    gen_gradient_steps_u8,
    gen_polygons_u16,
    gen_mosaic_f32,
    gen_checker_u8,
    gen_random,
)
