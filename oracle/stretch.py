"""asinh gray-scale stretch and its derivatives, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2.6 of the paper maps pixel values to new gray levels with per-pixel
functions (linear, logarithmic, exponential, power law) before they are fed
to neural networks.  The stretch here is y = b * asinh(v / a) with softening
a > 0 and scale b, which is logarithmic for |v| >> a and linear near 0:

  dy/dv = b / sqrt(a^2 + v^2)
  dy/da = -b v / (a sqrt(a^2 + v^2))
  dy/db = asinh(v / a)
"""
from __future__ import annotations

import math

import numpy as np


def asinh_forward(v, a: float, b: float) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return b * np.arcsinh(v / a)


def asinh_backward(v, g, a: float, b: float):
    """Given upstream g = dL/dy: (dL/dv, dL/da, dL/db); the scalar sums are
    exact and rounded once."""
    v = np.asarray(v, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    root = np.sqrt(a * a + v * v)
    dv = g * (b / root)
    da = math.fsum((g * (-b * v / (a * root))).ravel().tolist())
    db = math.fsum((g * np.arcsinh(v / a)).ravel().tolist())
    return dv, da, db
