"""Pins of the photometry oracle (Sec. 2.2.5, aperture photometry): disk
areas, numerical quadrature, closed-form fluxes, finite differences."""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

from oracle import Params
from oracle import photometry as ph
from oracle.params import SRC_APERTURE_OFF_EDGE, SRC_NO_SKY


def _weights(cx, cy, r):
    tot = 0.0
    out = {}
    for py in ph.window(cy, r):
        for px in ph.window(cx, r):
            w = ph.overlap(cx, cy, r, px, py)
            out[(px, py)] = w
            tot += w
    return out, tot


@pytest.mark.parametrize("r", [0.3, 1.0, 2.7, 5.0, 8.0, 12.0])
def test_weights_sum_to_disk_area(r):
    rng = np.random.default_rng(int(r * 10))
    for _ in range(5):
        cx, cy = rng.uniform(20, 30, 2)
        _, tot = _weights(cx, cy, r)
        assert tot == pytest.approx(math.pi * r * r, rel=1e-13)
        w, _ = _weights(cx, cy, r)
        assert all(-1e-13 <= v <= 1 + 1e-13 for v in w.values())


def test_small_disks():
    # r <= 1/2 centred on a pixel centre lies in one pixel
    assert ph.overlap(10.0, 7.0, 0.3, 10, 7) == pytest.approx(
        math.pi * 0.09, rel=1e-14)
    assert ph.overlap(10.0, 7.0, 0.5, 10, 7) == pytest.approx(
        math.pi / 4, rel=1e-14)
    assert ph.overlap(10.0, 7.0, 0.5, 11, 7) == pytest.approx(0.0, abs=1e-15)
    # centred on a pixel corner: a quarter disk in each of four pixels
    for px, py in ((3, 3), (4, 3), (3, 4), (4, 4)):
        assert ph.overlap(3.5, 3.5, 0.8, px, py) == pytest.approx(
            math.pi * 0.64 / 4, rel=1e-14)


def _quad_overlap(cx, cy, r, px, py):
    # integrate the chord length of the disk inside the pixel's y-range
    def chord(x):
        if abs(x - cx) >= r:
            return 0.0
        h = math.sqrt(r * r - (x - cx) ** 2)
        lo, hi = max(py - 0.5, cy - h), min(py + 0.5, cy + h)
        return max(0.0, hi - lo)
    a, b = px - 0.5, px + 0.5
    pts = [x for x in (cx - r, cx + r) if a < x < b]
    val, _ = scipy.integrate.quad(chord, a, b, points=pts or None,
                                  epsabs=1e-12, epsrel=1e-12, limit=400)
    return val


def test_overlap_matches_quadrature():
    rng = np.random.default_rng(11)
    for _ in range(40):
        r = rng.uniform(0.4, 6.0)
        cx, cy = rng.uniform(-2, 2, 2)
        px, py = rng.integers(-7, 8, 2)
        assert ph.overlap(cx, cy, r, int(px), int(py)) == pytest.approx(
            _quad_overlap(cx, cy, r, int(px), int(py)), abs=2e-9)


def test_overlap_gradient_matches_finite_difference():
    rng = np.random.default_rng(12)
    h = 1e-6
    for _ in range(60):
        r = rng.uniform(0.7, 6.0)
        cx, cy = rng.uniform(-1, 1, 2)
        px, py = rng.integers(-6, 7, 2)
        gx, gy = ph.overlap_grad(cx, cy, r, int(px), int(py))
        fx = (ph.overlap(cx + h, cy, r, px, py)
              - ph.overlap(cx - h, cy, r, px, py)) / (2 * h)
        fy = (ph.overlap(cx, cy + h, r, px, py)
              - ph.overlap(cx, cy - h, r, px, py)) / (2 * h)
        assert gx == pytest.approx(fx, abs=2e-7)
        assert gy == pytest.approx(fy, abs=2e-7)


def test_constant_image_zero_flux():
    img = np.full((60, 60), 1234.0, dtype=np.float32)
    B = np.zeros_like(img)
    r = ph.measure(img, B, 29.3, 30.1, Params())
    assert r["sky"] == pytest.approx(1234.0, rel=1e-14)
    assert r["area_ap"] == pytest.approx(25 * math.pi, rel=1e-13)
    assert r["area_ann"] == pytest.approx(80 * math.pi, rel=1e-13)
    assert r["flux"] == pytest.approx(0.0, abs=1e-8)
    assert r["flags"] == 0


def test_plane_image_centred_disk():
    # a symmetric disk about a pixel centre or corner averages a plane
    # to its value at the centre
    y, x = np.mgrid[0:64, 0:64]
    img = (300.0 + 2.0 * x - 1.5 * y).astype(np.float32)
    B = np.zeros_like(img)
    p = Params(sky_clip_iters=0)
    for cx, cy in ((31.0, 33.0), (31.5, 32.5)):
        r = ph.measure(img, B, cx, cy, p)
        c = 300.0 + 2.0 * cx - 1.5 * cy
        assert r["sky"] == pytest.approx(c, rel=1e-13)
        raw = r["flux"] + r["sky"] * r["area_ap"]
        assert raw == pytest.approx(c * 25 * math.pi, rel=1e-13)


def test_gaussian_star_enclosed_flux():
    sig, F = 3.0 / 2.3548200450309493, 1e5
    cx, cy = 40.3, 38.7
    y, x = np.mgrid[0:80, 0:80].astype(np.float64)
    c = 1 / (sig * math.sqrt(2))
    gx = 0.5 * (scipy.special.erf((x + 0.5 - cx) * c)
                - scipy.special.erf((x - 0.5 - cx) * c))
    gy = 0.5 * (scipy.special.erf((y + 0.5 - cy) * c)
                - scipy.special.erf((y - 0.5 - cy) * c))
    img = (500.0 + F * gx * gy).astype(np.float32)
    r = ph.measure(img, np.zeros_like(img), cx, cy, Params())
    want = F * (1 - math.exp(-25 / (2 * sig * sig)))
    # pixel values are integrals over whole pixels, weights are area
    # fractions: equal only up to the pixel discretisation (~1e-3 here)
    assert r["flux"] == pytest.approx(want, rel=1e-3)


def test_edge_and_no_sky_flags():
    img = np.full((20, 20), 5.0, dtype=np.float32)
    r = ph.measure(img, np.zeros_like(img), 1.0, 10.0, Params())
    assert r["flags"] & SRC_APERTURE_OFF_EDGE
    img[:] = np.nan
    img[10, 10] = 5.0
    r = ph.measure(img, np.zeros_like(img), 10.0, 10.0, Params())
    assert r["flags"] & SRC_NO_SKY and r["sky"] == 0.0


def _noisy_star(seed=13):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:48, 0:48].astype(np.float64)
    cx, cy = 23.6, 24.2
    img = 200 + 4e4 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / 4.5)
    img = (img + rng.normal(0, 5, img.shape)).astype(np.float32)
    return img, cx + 0.2, cy - 0.3


def test_adjoint_pixels_exact_linear():
    img, cx, cy = _noisy_star()
    B = np.zeros_like(img)
    p = Params()
    r = ph.measure(img, B, cx, cy, p)
    gv, _, _ = ph.measure_adjoint(img, B, cx, cy, p, r["sky_pixels"])
    # flux is linear in v when the sky mask is held fixed: check with
    # a perturbation small enough to keep the mask
    for (px, py) in [(23, 24), (14, 24), (33, 24)] + list(gv)[::37]:
        img2 = img.copy()
        img2[py, px] += np.float32(0.25)
        r2 = ph.measure(img2, B, cx, cy, p)
        if sorted(r2["sky_pixels"]) != sorted(r["sky_pixels"]):
            continue
        d = (r2["flux"] - r["flux"]) / (float(img2[py, px]) -
                                         float(img[py, px]))
        assert d == pytest.approx(gv.get((px, py), 0.0), abs=1e-7)


def test_adjoint_centre_matches_finite_difference():
    img, cx, cy = _noisy_star()
    B = np.zeros_like(img)
    p = Params()
    r = ph.measure(img, B, cx, cy, p)
    _, gx, gy = ph.measure_adjoint(img, B, cx, cy, p, r["sky_pixels"])
    h = 1e-3
    def f(ax, ay):
        return _flux_fixed_mask(img, B, ax, ay, p, r["sky_pixels"])
    fx = (f(cx + h, cy) - f(cx - h, cy)) / (2 * h)
    fy = (f(cx, cy + h) - f(cx, cy - h)) / (2 * h)
    assert gx == pytest.approx(fx, rel=1e-4, abs=1e-3)
    assert gy == pytest.approx(fy, rel=1e-4, abs=1e-3)


def _flux_fixed_mask(img, B, cx, cy, p, sky_pixels):
    keep = set(sky_pixels)
    h, w = img.shape
    num = den = ap = raw = 0.0
    for py in ph.window(cy, p.r_out):
        for px in ph.window(cx, p.r_out):
            if not (0 <= px < w and 0 <= py < h):
                continue
            v = float(img[py, px]) - float(B[py, px])
            wa = ph.overlap(cx, cy, p.r_ap, px, py)
            wn = (ph.overlap(cx, cy, p.r_out, px, py)
                  - ph.overlap(cx, cy, p.r_in, px, py))
            ap += wa
            raw += wa * v
            if (px, py) in keep:
                num += wn * v
                den += wn
    return raw - (num / den) * ap


def test_symmetric_star_zero_centre_gradient():
    y, x = np.mgrid[0:41, 0:41].astype(np.float64)
    img = (100 + 1e4 * np.exp(-((x - 20) ** 2 + (y - 20) ** 2) / 3.0))
    img = img.astype(np.float32)
    B = np.zeros_like(img)
    p = Params()
    r = ph.measure(img, B, 20.0, 20.0, p)
    _, gx, gy = ph.measure_adjoint(img, B, 20.0, 20.0, p, r["sky_pixels"])
    assert abs(gx) < 1e-8 and abs(gy) < 1e-8
