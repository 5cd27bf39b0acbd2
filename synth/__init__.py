"""Seeded synthetic astronomical frames.

This package only draws inputs: sky levels and gradients, point sources,
photon and read noise, cosmic-ray hits, dead columns and saturation.  It holds
no step of the pre-processing method itself (no background statistics,
thresholds, labelling or photometry), so the CPU oracle and the GPU path can
both take their inputs from it without sharing any of the method's arithmetic.
"""
from .frames import (FrameSpec, spec_for, config_frame_specs, render,
                     make_frame, CONFIG_NAMES)

__all__ = ["FrameSpec", "spec_for", "config_frame_specs", "render",
           "make_frame", "CONFIG_NAMES"]
