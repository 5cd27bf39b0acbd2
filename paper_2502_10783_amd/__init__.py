"""MI355X-native astronomical image pre-processing hot path.

HIP kernels for gfx950 behind the C ABI of include/ipp.h (libipp.so):
background estimation (mesh of sigma-clipped statistics, median filter,
spline), detection with connected-component labelling and pre-analysis,
and aperture photometry, per frame or as a fused batch; gray-scale
transformations (zscale, point maps, histogram equalization, asinh).
"""
from ._lib import lib, LIB_PATH, header_functions  # noqa: F401
from ._lib import (IPP_MAP_LINEAR, IPP_MAP_LOG, IPP_MAP_EXP,  # noqa: F401
                   IPP_MAP_POWER)
from .api import (Params, DeblendParams, SubtractParams, Context,  # noqa
                  SourceTable, IppError)
from .autograd import ApertureFlux, AsinhStretch, refine_centroids  # noqa

__all__ = ["Params", "DeblendParams", "SubtractParams", "Context", "SourceTable", "IppError", "lib",
           "LIB_PATH", "header_functions", "ApertureFlux", "AsinhStretch",
           "refine_centroids", "IPP_MAP_LINEAR", "IPP_MAP_LOG",
           "IPP_MAP_EXP", "IPP_MAP_POWER"]
