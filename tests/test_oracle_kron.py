"""Pins of the AUTO (Kron) photometry oracle (Sec. 2.2.5 per-object
photometry; Sec. 3.3 compares auto magnitudes): the exact ellipse-pixel
overlap against the circle overlap of the aperture photometry (another
method) and adaptive quadrature, total area, mirror symmetry; the Kron
radius on a hand-worked image; exact totals of a top-hat source; flags."""
import math

import numpy as np
import pytest
import scipy.integrate

from oracle import kron as kr
from oracle import photometry as oph


def test_circular_case_equals_the_circle_overlap():
    # x2 = y2 = s - 1/12, xy = 0: q = (dx^2 + dy^2) / s, so q <= R^2 is the
    # disk of radius R sqrt(s), whose overlaps the aperture photometry
    # computes by quadrant areas
    s = 2.25
    sh = kr.shape(s - 1.0 / 12.0, s - 1.0 / 12.0, 0.0)
    R = 2.0
    r = R * math.sqrt(sh[0])
    cx, cy = 10.3, 7.8
    for py in range(3, 13):
        for px in range(5, 16):
            a = kr.ellipse_overlap(sh, R, cx, cy, px, py)
            b = oph.overlap(cx, cy, r, px, py)
            assert abs(a - b) <= 1e-12, (px, py, a, b)


def _quad_overlap(sh, R, cx, cy, px, py):
    """Area of pixel (px, py) inside q <= R^2 by adaptive quadrature of the
    vertical chord length."""
    X, Y, xy, det = sh

    def chord(x):
        dx = x - cx
        # q(dx, dy) <= R^2 in dy: (X / det) dy^2 - (2 xy dx / det) dy
        # + (Y dx^2 / det - R^2) <= 0
        a = X / det
        b = -2.0 * xy * dx / det
        c = Y * dx * dx / det - R * R
        disc = b * b - 4 * a * c
        if disc <= 0:
            return 0.0
        r0 = (-b - math.sqrt(disc)) / (2 * a) + cy
        r1 = (-b + math.sqrt(disc)) / (2 * a) + cy
        lo, hi = max(r0, py - 0.5), min(r1, py + 0.5)
        return max(hi - lo, 0.0)

    v, _ = scipy.integrate.quad(chord, px - 0.5, px + 0.5, epsabs=1e-13,
                                epsrel=1e-13, limit=200)
    return v


def test_overlap_by_quadrature():
    sh = kr.shape(3.1, 1.2, 0.9)
    R, cx, cy = 1.7, 20.4, 11.1
    n = 0
    for py in range(6, 17):
        for px in range(14, 27):
            a = kr.ellipse_overlap(sh, R, cx, cy, px, py)
            if 0.0 < a < 1.0:
                n += 1
                b = _quad_overlap(sh, R, cx, cy, px, py)
                assert abs(a - b) <= 1e-9, (px, py, a, b)
    assert n > 10


def test_total_area_and_mirror_symmetry():
    sh = kr.shape(4.0, 2.0, -1.3)
    R, cx, cy = 2.6, 30.0, 25.0
    X, Y, xy, det = sh
    tot = 0.0
    w = {}
    for py in range(10, 41):
        for px in range(15, 46):
            w[px, py] = kr.ellipse_overlap(sh, R, cx, cy, px, py)
            tot += w[px, py]
    assert abs(tot - math.pi * R * R * math.sqrt(det)) <= 1e-10
    mir = kr.shape(4.0, 2.0, 1.3)      # xy -> -xy: mirror in x
    for (px, py), a in w.items():
        b = kr.ellipse_overlap(mir, R, cx, cy, int(2 * cx) - px, py)
        assert abs(a - b) <= 1e-12


def test_kron_radius_hand_worked():
    # two pixels of value 1 at q = 0 and q = 9 (x2 = y2 = 11/12, so
    # X = Y = 1 up to rounding): r1 = (0 * 1 + 3 * 1) / 2 = 1.5 and
    # R = 2.5 * 1.5 = 3.75 > 3.5
    img = np.zeros((40, 40), dtype=np.float32)
    B = np.zeros_like(img)
    img[20, 20] = 1.0
    img[20, 23] = 1.0
    R, f, a, fl = kr.auto_one(img, B, 20.0, 20.0, 11 / 12, 11 / 12, 0.0)
    assert abs(R - 3.75) <= 1e-12 and fl == 0
    # the ellipse of radius 3.75 (a disk) holds both pixels whole
    assert f == 2.0
    # a pixel at q = 1 instead: r1 = 0.5, R = max(1.25, 3.5) = 3.5
    img[20, 23] = 0.0
    img[20, 21] = 1.0
    R, f, a, fl = kr.auto_one(img, B, 20.0, 20.0, 11 / 12, 11 / 12, 0.0)
    assert abs(R - 3.5) <= 1e-15 and fl == 0
    # no positive light: the minimum radius, flagged
    R, f, a, fl = kr.auto_one(-img, B, 20.0, 20.0, 11 / 12, 11 / 12, 0.0)
    assert R == 3.5 and fl & kr.AUTO_RMIN


def test_top_hat_source_total_flux_and_constant_image():
    h = w = 64
    y, x = np.mgrid[0:h, 0:w]
    disk = ((x - 32) ** 2 + (y - 31) ** 2) <= 16
    img = np.where(disk, 50.0, 0.0).astype(np.float32)
    B = np.zeros_like(img)
    # the top hat's own moments (x2 = y2 = 4.0 roughly): R >= 3.5 gives an
    # ellipse of radius >= 3.5 * 2.06 > 4.5, holding every disk pixel
    xs, ys = x[disk], y[disk]
    x2 = float(np.mean((xs - 32.0) ** 2))
    R, f, a, fl = kr.auto_one(img, B, 32.0, 31.0, x2, x2, 0.0)
    assert f == 50.0 * disk.sum() and fl == 0
    X = x2 + 1 / 12
    assert abs(a - math.pi * R * R * X) <= 1e-9
    # a constant image: flux = constant * area
    c = np.full((h, w), 7.0, dtype=np.float32)
    R, f, a, fl = kr.auto_one(c, B, 30.3, 29.6, 2.0, 1.5, 0.4)
    assert abs(f - 7.0 * a) <= 1e-9 * f


def test_flags():
    img = np.ones((30, 30), dtype=np.float32)
    B = np.zeros_like(img)
    R, f, a, fl = kr.auto_one(img, B, 1.0, 15.0, 2.0, 2.0, 0.0)
    assert fl & kr.AUTO_OFF_EDGE
    R, f, a, fl = kr.auto_one(img, B, 15.0, 15.0, math.nan, 2.0, 0.0)
    assert fl == kr.AUTO_BAD_SHAPE and math.isnan(f)
    # a degenerate shape (det <= 0 after regularisation is impossible for
    # valid moments; forced with |xy| > sqrt(X Y))
    R, f, a, fl = kr.auto_one(img, B, 15.0, 15.0, 1.0, 1.0, 2.0)
    assert fl == kr.AUTO_BAD_SHAPE


def test_min_q_is_the_minimum_over_the_square():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x2, y2 = rng.uniform(0.2, 5.0, 2)
        xy = rng.uniform(-0.9, 0.9) * math.sqrt(x2 * y2)
        sh = kr.shape(x2, y2, xy)
        x0, y0 = rng.uniform(-4, 4, 2)
        x1, y1 = x0 + 1.0, y0 + 1.0
        g = np.linspace(0, 1, 201)
        gx, gy = np.meshgrid(x0 + g, y0 + g)
        brute = np.min([kr.qform(sh, a, b) for a, b in
                        zip(gx.ravel(), gy.ravel())])
        m = kr.min_q(sh, x0, x1, y0, y1)
        assert m <= brute + 1e-12
        assert m >= brute - 1e-3 * (1 + brute)
