"""Seeded synthetic inputs for window matching (stand-ins for serial-section EM data).

This module only makes inputs: textures, membrane-like curves, warps and noise.
It holds none of the matching method's arithmetic, so both the FP64 oracle side
(tests) and the HIP path (tests, bench) can consume the same bytes.
"""
from .synth import (  # noqa: F401
    make_pair64,
    make_section,
    make_section_pair,
    make_stack,
    random_affine_about_center,
    warp_affine,
    window_grid,
    config4_thetas,
)
