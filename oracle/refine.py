"""Gradient-based centroid refinement, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's photometry measures each object at its detected position
(Sec. 2.2.5); this library adds a differentiable photometry so positions can
be refined by gradients.  The rule (this library's reading; the paper has
none): maximise J(c) = F_rc(c) / F_ap(c0), the sky-subtracted flux in an
aperture of radius r_c (default 2 px) normalised by the flux in the default
aperture at the starting point, by `steps` plain ascent steps
c <- c + eta * dJ/dc (eta = 3 px^2), the gradient taken with the sky clip
mask of the current forward held fixed.  Sources with F_ap(c0) <= 0 stay.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .params import Params
from .photometry import measure, measure_adjoint


def refine_centroids(frame, B32, xs, ys, p: Params, steps: int = 10,
                     eta: float = 3.0, r_c: float = 2.0):
    img = np.asarray(frame, dtype=np.float32)
    B = np.asarray(B32, dtype=np.float32)
    x = np.array(xs, dtype=np.float64)
    y = np.array(ys, dtype=np.float64)
    pc = replace(p, r_ap=r_c)
    for k in range(x.size):
        f0 = measure(img, B, float(x[k]), float(y[k]), p)["flux"]
        if not f0 > 0:
            continue
        for _ in range(steps):
            r = measure(img, B, float(x[k]), float(y[k]), pc)
            _, gx, gy = measure_adjoint(img, B, float(x[k]), float(y[k]), pc,
                                        r["sky_pixels"], 1.0 / f0)
            x[k] += eta * gx
            y[k] += eta * gy
    return x, y
