"""Pins of the detection oracle (Sec. 2.2.5): hand-worked labellings,
scipy's labelling, closed-form pre-analysis and exact rational sums."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage

from oracle import Params
from oracle import detect as dt
from oracle.params import SRC_INEXACT_SUM_RANGE, SRC_NONPOSITIVE_FLUX

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _patterns():
    out = []
    with open(os.path.join(GOLDEN, "ccl_patterns.txt")) as f:
        lines = [ln.rstrip("\n") for ln in f if not ln.startswith("#")]
    i = 0
    while i < len(lines):
        if not lines[i].startswith("pattern"):
            i += 1
            continue
        _, name, conn, area = lines[i].split()
        i += 1
        mask = []
        while lines[i] != "labels":
            mask.append([c == "x" for c in lines[i]])
            i += 1
        i += 1
        lab = []
        while i < len(lines) and not lines[i].startswith("pattern"):
            if lines[i].strip():
                lab.append([int(c) for c in lines[i]])
            i += 1
        out.append((name, int(conn), int(area), np.array(mask),
                    np.array(lab)))
    return out


@pytest.mark.parametrize("case", _patterns(), ids=lambda c: f"{c[0]}-{c[1]}")
def test_golden_patterns(case):
    name, conn, area, mask, want = case
    lab, n = dt.label_components(mask, conn)
    lab, n = dt.apply_min_area(lab, n, area)
    assert np.array_equal(lab, want), name
    assert n == want.max()


@pytest.mark.parametrize("density", [0.07, 0.41, 0.6])
@pytest.mark.parametrize("conn", [4, 8])
def test_labels_equal_scipy(density, conn):
    rng = np.random.default_rng(int(density * 100) + conn)
    mask = rng.random((97, 131)) < density
    lab, n = dt.label_components(mask, conn)
    st = np.ones((3, 3)) if conn == 8 else None
    ref, nref = scipy.ndimage.label(mask, structure=st)
    assert n == nref
    assert np.array_equal(lab, ref)        # scipy numbers in scan order too


def test_component_spanning_frame_and_spiral():
    h, w = 41, 53
    sp = np.zeros((h, w), dtype=bool)
    y0, y1, x0, x1 = 0, h - 1, 0, w - 1
    while y0 <= y1 and x0 <= x1:            # square spiral, 1-px walls
        sp[y0, x0:x1 + 1] = True
        sp[y0:y1 + 1, x1] = True
        if y1 - 2 > y0:
            sp[y1, x0:x1 + 1] = True
        if x0 + 2 <= x1 and y0 + 2 <= y1:
            sp[y0 + 2:y1 + 1, x0] = True
        y0, x0, y1, x1 = y0 + 2, x0 + 2, y1 - 2, x1 - 2
    lab, n = dt.label_components(sp, 8)
    ref, nref = scipy.ndimage.label(sp, structure=np.ones((3, 3)))
    assert n == nref and np.array_equal(lab, ref)


def test_threshold_is_strict_and_finite_only():
    I = np.array([[10.0, 11.0, np.nan, np.inf, -np.inf]], dtype=np.float32)
    B = np.zeros_like(I)
    R = np.full_like(I, 10.0 / 1.5)
    det, v = dt.threshold(I, B, R, 1.5)
    t = 1.5 * np.float64(np.float32(10.0 / 1.5))
    assert det.tolist() == [[10.0 > t, True, False, False, False]]


def _src(I, B, p):
    det, _ = dt.threshold(I, B, np.zeros_like(B), 0.0)
    lab, n = dt.label_components(det, p.connectivity)
    lab, n = dt.apply_min_area(lab, n, p.min_area)
    return dt.source_table(I, B, lab, n)


def test_box_source_closed_form():
    I = np.full((12, 14), 1000.0, dtype=np.float32)
    B = np.full_like(I, 1000.0)
    I[3:6, 5:8] = 1010.0                   # 3x3 box, v = 10
    t = _src(I, B, Params(min_area=1))
    assert t["npix"].tolist() == [9]
    assert (t["xmin"][0], t["xmax"][0], t["ymin"][0], t["ymax"][0]) == \
        (5, 7, 3, 5)
    assert t["flux_iso"][0] == 90.0
    assert (t["x"][0], t["y"][0]) == (6.0, 4.0)
    assert (t["peak"][0], t["peak_x"][0], t["peak_y"][0]) == (10.0, 5, 3)


def test_l_shape_barycentre_rational():
    I = np.full((8, 8), 100.0, dtype=np.float32)
    B = np.full_like(I, 100.0)
    pix = {(2, 2): 3.0, (3, 2): 5.0, (4, 2): 7.0, (4, 3): 11.0, (4, 4): 2.5}
    for (y, x), v in pix.items():
        I[y, x] = 100.0 + v
    t = _src(I, B, Params(min_area=1))
    S = sum(Fraction(v) for v in pix.values())
    sx = sum(Fraction(v) * (x - 2) for (y, x), v in pix.items())
    sy = sum(Fraction(v) * (y - 2) for (y, x), v in pix.items())
    assert t["flux_iso"][0] == float(S)
    assert t["x"][0] == 2 + float(sx) / float(S)
    assert t["y"][0] == 2 + float(sy) / float(S)
    assert (t["peak_x"][0], t["peak_y"][0]) == (3, 4)


def test_exact_sum_rounded_once():
    # a sum that a sequential binary64 loop gets wrong
    I = np.zeros((1, 30), dtype=np.float32)
    B = np.zeros_like(I)
    I[0, :4] = 2.0 ** 24
    I[0, 4:] = np.float32(2.0 ** -5 * (1 + 3 * 2.0 ** -23))
    B[0, 4:] = np.float32(2.0 ** -5)
    t = _src(I, B, Params(min_area=1))
    vals = [Fraction(float(a)) - Fraction(float(b))
            for a, b in zip(I[0], B[0])]
    assert t["flux_iso"][0] == float(sum(vals))
    naive = 0.0
    for v in vals:
        naive += float(v)
    assert naive != float(sum(vals))
    assert t["flags"][0] == 0


def test_peak_tie_goes_to_lowest_raster_index():
    I = np.full((5, 5), 10.0, dtype=np.float32)
    B = np.zeros_like(I)
    I[1, 3] = I[2, 1] = 50.0
    t = _src(I, B, Params(min_area=1))
    assert (t["peak_x"][0], t["peak_y"][0]) == (3, 1)


def test_out_of_range_pixel_flags_row():
    I = np.full((3, 3), 1e-3, dtype=np.float32)     # below 2^-5
    B = np.zeros_like(I)
    t = _src(I, B, Params(min_area=1))
    assert t["flags"][0] & SRC_INEXACT_SUM_RANGE


def _moments_of(mask, dvals):
    """Moments of one candidate: image 1 + d on a unit sky, label 1."""
    I = np.ones(mask.shape, dtype=np.float32)
    I[mask] += np.asarray(dvals, dtype=np.float32)
    lab = mask.astype(np.int32)
    return dt.source_moments(I, np.ones_like(I), lab, 1)[0]


@pytest.mark.parametrize("w,h", [(5, 3), (4, 7), (6, 6), (1, 9)])
def test_moments_of_a_uniform_box(w, h):
    # discrete uniform: variance (n^2 - 1) / 12 along each axis, no xy
    m = np.zeros((12, 14), dtype=bool)
    m[2:2 + h, 3:3 + w] = True
    x2, y2, xy, a, b, th = _moments_of(m, 4.0)
    assert math.isclose(x2, (w * w - 1) / 12, rel_tol=1e-15, abs_tol=1e-15)
    assert math.isclose(y2, (h * h - 1) / 12, rel_tol=1e-15, abs_tol=1e-15)
    assert abs(xy) <= 1e-15
    big, small = max(x2, y2), min(x2, y2)
    assert math.isclose(a, math.sqrt(big), rel_tol=1e-15)
    assert math.isclose(b, math.sqrt(small), rel_tol=1e-15, abs_tol=1e-15)
    if w > h:
        assert th == 0.0
    elif h > w:
        assert math.isclose(th, math.pi / 2, rel_tol=1e-15)


def test_moments_of_a_diagonal_and_a_weighted_pair():
    n = 7
    m = np.zeros((10, 10), dtype=bool)
    m[np.arange(n) + 1, np.arange(n) + 2] = True
    x2, y2, xy, a, b, th = _moments_of(m, 3.0)
    v = (n * n - 1) / 12
    for got in (x2, y2, xy):
        assert math.isclose(got, v, rel_tol=1e-15)
    assert math.isclose(a, math.sqrt(2 * v), rel_tol=1e-15) and b == 0.0
    assert math.isclose(th, math.pi / 4, rel_tol=1e-15)
    # weights 1 and 2 at x = 0 and x = 3 (one row): mean 2, variance 2
    m = np.zeros((3, 6), dtype=bool)
    m[1, 1] = m[1, 4] = True
    x2, y2, xy, a, b, th = _moments_of(m, [1.0, 2.0])
    assert (x2, y2, xy, th) == (2.0, 0.0, 0.0, 0.0)
    assert a == math.sqrt(2.0) and b == 0.0


def test_moments_rotate_with_the_shape():
    m = np.zeros((9, 9), dtype=bool)
    m[2, 2:7] = True
    m[2:6, 2] = True
    m[5, 3] = True                                   # an irregular L
    rng = np.random.default_rng(5)
    d = rng.integers(1, 50, m.shape).astype(np.float32)
    x2, y2, xy, a, b, th = _moments_of(m, d[m])
    mr = np.rot90(m)                                 # (x, y) -> (y, -x)
    x2r, y2r, xyr, ar, br, _ = _moments_of(mr, np.rot90(d)[mr])
    assert math.isclose(x2r, y2, rel_tol=1e-12)
    assert math.isclose(y2r, x2, rel_tol=1e-12)
    assert math.isclose(xyr, -xy, rel_tol=1e-12)
    assert math.isclose(ar, a, rel_tol=1e-12) and math.isclose(br, b,
                                                              rel_tol=1e-12)


def test_nonpositive_flux_takes_the_unweighted_centroid():
    """Sec. 2.2.5 pre-analysis with a threshold below the sky (nsigma < 0):
    candidates whose values sum to <= 0 take the plain pixel mean as their
    centre and carry the flag (closed forms)."""
    B = np.full((8, 9), 100.0, dtype=np.float32)
    I = B - 100.0                       # v = -100: below t = -50
    for y, x in ((1, 1), (1, 2), (2, 1)):
        I[y, x] = 90.0                  # v = -10: detected, sum -30
    I[5, 5], I[5, 6], I[6, 6] = 105.0, 95.0, 100.0    # v = 5, -5, 0: sum 0
    R = np.full_like(B, 10.0)
    p = Params(min_area=1, det_nsigma=-5.0)
    d = dt.detect(I, B, R, p)
    t = d["table"]
    assert d["n"] == 2
    assert t["flux_iso"].tolist() == [-30.0, 0.0]
    assert t["x"][0] == 1.0 + 1.0 / 3.0 and t["y"][0] == 1.0 + 1.0 / 3.0
    assert t["x"][1] == 5.0 + 2.0 / 3.0 and t["y"][1] == 5.0 + 1.0 / 3.0
    assert all(f & SRC_NONPOSITIVE_FLUX for f in t["flags"])
    # peak: the largest value, the first of equal ones in raster order
    assert (t["peak"][0], t["peak_x"][0], t["peak_y"][0]) == (-10.0, 1, 1)
    assert (t["peak"][1], t["peak_x"][1], t["peak_y"][1]) == (5.0, 5, 5)


def test_huge_value_is_clamped_below_two_to_the_62():
    """A finite value whose fixed-point integer D = v 2^28 exceeds the
    int64 sum range is clamped to 2^62 - 1 (not 2^62) and flags the row."""
    I = np.full((4, 4), 1.0, dtype=np.float32)
    B = np.zeros_like(I)
    I[1, 2] = np.float32(1e11)          # v 2^28 ~ 2.7e19 > 2^62
    I[0, 0] = np.float32(2.0 ** 34)     # v 2^28 = 2^62 exactly: clamped too
    t = _src(I, B, Params(min_area=1))
    dmax = (1 << 62) - 1
    S = 2 * dmax + 14 * (1 << 28)
    assert t["flux_iso"][0] == float(Fraction(S, 1 << 28))
    Sx = dmax * 2 + dmax * 0 + sum((1 << 28) * x for x in range(4)
                                   for y in range(4)
                                   if (y, x) not in ((1, 2), (0, 0)))
    assert t["x"][0] == float(Sx) / float(S)
    assert t["flags"][0] & SRC_INEXACT_SUM_RANGE
