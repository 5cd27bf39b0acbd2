"""MI355X-native astronomical image pre-processing hot path.

HIP kernels for gfx950 behind the C ABI of include/ipp.h (libipp.so):
background estimation (mesh of sigma-clipped statistics, median filter,
spline), detection with connected-component labelling and pre-analysis,
and aperture photometry, per frame or as a fused batch.
"""
from ._lib import lib, LIB_PATH, header_functions  # noqa: F401
from .api import Params, Context, SourceTable, IppError  # noqa: F401
from .autograd import ApertureFlux, AsinhStretch, refine_centroids  # noqa

__all__ = ["Params", "Context", "SourceTable", "IppError", "lib",
           "LIB_PATH", "header_functions", "ApertureFlux", "AsinhStretch",
           "refine_centroids"]
