"""Pins of the oracle's centroid refinement: a noise-free Gaussian star
centred on a pixel centre (so its pixelated image is symmetric
about the true centre) is found from a 0.3 px offset; off-grid stars end on
a stationary point of the aperture flux; a centred star stays put."""
import numpy as np
import scipy.special

from oracle import Params
from oracle.refine import refine_centroids


def _star(cx, cy, fwhm=3.0, F=2e5, n=48, sky=1000.0):
    sig = fwhm / 2.3548200450309493
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    c = 1 / (sig * np.sqrt(2))
    gx = 0.5 * (scipy.special.erf((x + 0.5 - cx) * c)
                - scipy.special.erf((x - 0.5 - cx) * c))
    gy = 0.5 * (scipy.special.erf((y + 0.5 - cy) * c)
                - scipy.special.erf((y - 0.5 - cy) * c))
    img = (sky + F * gx * gy).astype(np.float32)
    return img, np.full_like(img, sky)


def test_converges_on_noise_free_symmetric_star():
    for cx, cy in ((24.0, 24.0), (17.0, 29.0)):
        img, B = _star(cx, cy)
        x0, y0 = np.array([cx + 0.3]), np.array([cy - 0.25])
        x, y = refine_centroids(img, B, x0, y0, Params(), steps=10)
        e0 = np.hypot(x0 - cx, y0 - cy)[0]
        e1 = np.hypot(x - cx, y - cy)[0]
        assert e1 < e0 / 50, (cx, cy, e0, e1)


def test_off_grid_star_ends_on_stationary_point():
    from oracle.photometry import measure, measure_adjoint
    from dataclasses import replace
    cx, cy = 23.37, 24.81
    img, B = _star(cx, cy)
    x, y = refine_centroids(img, B, np.array([cx + 0.3]),
                            np.array([cy - 0.25]), Params(), steps=40)
    pc = replace(Params(), r_ap=2.0)
    r = measure(img, B, x[0], y[0], pc)
    _, gx, gy = measure_adjoint(img, B, x[0], y[0], pc, r["sky_pixels"])
    r0 = measure(img, B, cx + 0.3, cy - 0.25, pc)
    _, gx0, gy0 = measure_adjoint(img, B, cx + 0.3, cy - 0.25, pc,
                                  r0["sky_pixels"])
    assert np.hypot(gx, gy) < 1e-6 * np.hypot(gx0, gy0)
    assert np.hypot(x[0] - cx, y[0] - cy) < 0.2


def test_centred_star_stays():
    img, B = _star(24.0, 24.0)
    x, y = refine_centroids(img, B, np.array([24.0]), np.array([24.0]),
                            Params(), steps=3)
    assert abs(x[0] - 24.0) < 1e-9 and abs(y[0] - 24.0) < 1e-9


def test_nonpositive_normaliser_leaves_source():
    img = np.full((40, 40), 100.0, dtype=np.float32)
    B = np.full_like(img, 100.0)
    x, y = refine_centroids(img, B, np.array([20.3]), np.array([19.6]),
                            Params(), steps=2)
    assert x[0] == 20.3 and y[0] == 19.6
