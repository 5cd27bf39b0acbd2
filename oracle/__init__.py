"""Plain, slow FP64 CPU oracle of the pre-processing hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code, table or helper
with the HIP implementation; the only common inputs are the seeded frames
from the ``synth`` package.

Each module follows a part of the paper (arXiv 2502.10783, "Image
Pre-Processing Framework for Time-Domain Astronomy in the Artificial
Intelligence Era"):

* ``background`` -- Sec. 2.2.2 (Background Estimation and Removal Function):
  mesh tiling, the median/mean/"sigma"/mode estimators of Eq. 1-4, the
  iterative sigma clipping, the median filter and the spline interpolation.
* ``detect``     -- Sec. 2.2.5 (Source Detection Function): pixel detection
  above a threshold, connection of pixels into candidates, and the
  pre-analysis of each candidate (peak value and total flux).
* ``deblend``    -- Sec. 2.2.5: multi-threshold deblending of the
  candidates into objects, and cleaning.
* ``kron``       -- Sec. 2.2.5: AUTO (Kron) photometry, the Kron radius
  and an exact ellipse-pixel overlap.
* ``subtract``   -- Sec. 2.2.4 (Image Subtraction Function): the
  spatially varying stamp convolution of Eq. 8-10 and the difference image
  (the kernel fit is not part of this path).
* ``photometry`` -- Sec. 2.2.5, last paragraph: per-object aperture
  photometry, with exact circle/pixel overlaps and a local sky annulus, and
  its adjoint (gradients with the sky clip mask held fixed).
* ``stretch``    -- Sec. 2.2.6 (Gray Scale Transformation Function): an asinh
  gray-scale map and its derivatives.
* ``gray``       -- Sec. 2.2.6: the zscale display range, linear /
  logarithmic / exponential / power-law maps and histogram equalization.
* ``refine``     -- gradient-ascent centroid refinement on the photometry
  adjoint (an addition to the paper's method).

Where the paper leaves a step open, the reading taken is stated in the
docstring of the function that implements it.  Every floating-point value is
IEEE binary64; sums that decide results are exact (``math.fsum`` or Python
integers) and rounded once.
"""
from .params import Params
from . import (background, detect, deblend, kron, photometry, stretch,
               refine, gray, subtract)

__all__ = ["Params", "background", "detect", "photometry", "stretch",
           "refine", "gray", "deblend", "kron", "subtract"]
