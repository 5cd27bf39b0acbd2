"""Pins of the deblending and cleaning oracle (Sec. 2.2.5, deblending and
cleaning phases): closed-form levels, hand-worked splits of small strips,
the contrast criterion on both sides of its bound, a cleaning merge worked
by hand, mirror symmetry, and partition invariants on random blends."""
import math

import numpy as np
import pytest

import oracle
from oracle import deblend as db
from oracle import detect as dt
from oracle.params import SRC_BLENDED


def test_levels_closed_form():
    # peak / t0 = 2^32 and 32 levels: five square roots give q = 2 exactly
    lv = db.levels(1.0, 2.0 ** 32, 32)
    assert lv == [2.0 ** i for i in range(1, 32)]
    # 4 levels of 3 -> 48: q = 2
    assert db.levels(3.0, 48.0, 4) == [6.0, 12.0, 24.0]
    lv = db.levels(1.5, 700.0, 32)
    assert len(lv) == 31 and all(a < b for a, b in zip(lv, lv[1:]))
    assert 1.5 < lv[0] and lv[-1] < 700.0
    assert abs(lv[-1] * (700.0 / 1.5) ** (1 / 32) - 700.0) < 1e-9


def _strip(values, params, B=100.0, R=None, nsigma=None):
    """One candidate along a 1-pixel strip inside a 3-row frame of value B
    (background B, rms R): returns the object labels along the strip and the
    oracle's result."""
    v = np.asarray(values, dtype=np.float64)
    w = v.size + 2
    I = np.full((3, w), B - 1000.0, dtype=np.float32)
    I[1, 1:-1] = (B + v).astype(np.float32)
    Bm = np.full_like(I, B)
    Rm = np.full_like(I, 1.0 if R is None else R)
    p = params
    det = dt.detect(I, Bm, Rm, p)
    assert det["n"] == 1
    out = db.deblend(I, Bm, Rm, det["labels"], det["table"], p)
    return out["objects"][1, 1:-1].tolist(), out


def test_two_equal_peaks_split_and_tie_goes_to_the_first():
    # t0 = 2 (nsigma 2, rms 1); two levels: q = sqrt(10 / 2), t1 = 4.47.
    # Above t1: pixels 1 and 5, two components each of intensity
    # 10 - 4.47 = 5.53 > 0.005 * 34.5: the candidate splits.  The seeds are
    # single pixels of equal flux and scale, so every other pixel goes to
    # the nearer seed, and pixel 3 (equidistant) to the first.
    p = oracle.Params(min_area=1, det_nsigma=2.0, deblend_nthresh=2)
    objs, out = _strip([3, 10, 3, 2.5, 3, 10, 3], p)
    assert objs == [1, 1, 1, 1, 2, 2, 2]
    assert out["n"] == 2 and out["counts"].tolist() == [2]
    t = out["table"]
    assert t["npix"].tolist() == [4, 3]
    assert t["flux_iso"].tolist() == [18.5, 16.0]
    assert t["parent"].tolist() == [1, 1]
    assert all(f & SRC_BLENDED for f in t["flags"])


def test_single_peak_is_not_split():
    p = oracle.Params(min_area=1, det_nsigma=2.0)
    objs, out = _strip([2.5, 4, 9, 30, 9, 4, 2.5], p)
    assert objs == [1] * 7 and out["n"] == 1
    assert not (out["table"]["flags"][0] & SRC_BLENDED)


def test_contrast_criterion_on_both_sides():
    # t0 = 2; with 2 levels t1 = 2 sqrt(50) = 14.14.  Above t1: the bright
    # pixel (100, intensity 85.86) and the faint one (v = 15, intensity
    # 0.858).  Root flux 100 + 15 + 3 * 2.5 = 122.5: the faint branch is
    # significant for mincont 0.005 (0.6125) and not for 0.01 (1.225).
    vals = [2.5, 100, 2.5, 15, 2.5]
    p = oracle.Params(min_area=1, det_nsigma=2.0, deblend_nthresh=2,
                      deblend_clean=False)
    objs, _ = _strip(vals, p)
    assert objs == [1, 1, 1, 2, 2]
    p.deblend_mincont = 0.01
    objs, _ = _strip(vals, p)
    assert objs == [1] * 5


def test_cleaning_merges_a_bump_in_a_bright_wing():
    # A bright pixel F at x = 0 and a bump peaking at 40 at x = 4; t0 = 2
    # (nsigma 2, rms 1), 4 levels: q = (F / 2)^(1/4).
    # F = 1e5: t1 = 2 * 50000^(1/4) = 29.9, above it {0} and {4}; the bump's
    # intensity 40 - 29.9 = 10.1 exceeds 1e-5 * 100058: the candidate splits.
    # Both seeds are single pixels (s2 = 1/6).  Pixel 3 (v = 4) scores
    # 1e5 / 6 / (1/6 + 9)^2 = 198 for the bright seed and 40 / 6 /
    # (1/6 + 1)^2 = 4.9 for the bump, so it and every other pixel but x = 4
    # go to the bright object.
    vals = [1e5, 3, 2.2, 4, 40, 4, 2.1]
    p = oracle.Params(min_area=1, det_nsigma=2.0, deblend_nthresh=4,
                      deblend_mincont=1e-5, deblend_clean=False)
    objs, _ = _strip(vals, p)
    assert objs == [1, 1, 1, 1, 2, 1, 1]
    # Cleaning: the bump object {4} has mean 40; the bright seed puts
    # 1e5 / 6 / (pi (1/6 + 16)^2) = 20.3 at x = 4; 40 - 20.3 > 2: it stays.
    p.deblend_clean = True
    objs, out = _strip(vals, p)
    assert objs == [1, 1, 1, 1, 2, 1, 1] and out["n"] == 2
    # F = 2e5: t1 = 35.6, the bump still splits off (intensity 4.4 > 2.0),
    # but the bright seed now puts 40.6 at x = 4: 40 - 40.6 < 2, merged.
    vals[0] = 2e5
    objs, out = _strip(vals, p)
    assert objs == [1] * 7 and out["n"] == 1
    # one object survives: it is not flagged as a split product
    assert not (out["table"]["flags"][0] & SRC_BLENDED)
    p.deblend_clean = False
    objs, _ = _strip(vals, p)
    assert objs == [1, 1, 1, 1, 2, 1, 1]


def _gauss_pair(sep, flux=(5e3, 5e3), size=41, fwhm=2.5):
    s = fwhm / (2 * math.sqrt(2 * math.log(2)))
    y, x = np.mgrid[0:size, 0:size].astype(np.float64)
    c = (size - 1) / 2
    img = np.full((size, size), 100.0)
    pos = [(c - sep / 2, c), (c + sep / 2, c)]
    for (xc, yc), f in zip(pos, flux):
        img += f / (2 * math.pi * s * s) * np.exp(
            -((x - xc) ** 2 + (y - yc) ** 2) / (2 * s * s))
    if flux[0] == flux[1]:
        # exactly mirror-symmetric in x (a + b == b + a)
        img = (img + img[:, ::-1]) / 2
    return img.astype(np.float32), pos


def test_mirror_symmetric_pair_gives_mirror_objects():
    img, pos = _gauss_pair(6.0)
    B = np.full_like(img, 100.0)
    R = np.full_like(img, 1.0)
    p = oracle.Params(det_nsigma=5.0)
    det = dt.detect(img, B, R, p)
    assert det["n"] == 1
    out = db.deblend(img, B, R, det["labels"], det["table"], p)
    assert out["n"] == 2
    o = out["objects"]
    # mirror in x about the centre column: object 1 <-> 2 off that column
    # (on it the two models tie in exact arithmetic; their rounded
    # barycentres decide)
    c = img.shape[1] // 2
    m = o[:, ::-1]
    left, right = o[:, :c], m[:, :c]
    assert np.array_equal(left == 1, right == 2)
    assert np.all(np.isin(o[:, c][o[:, c] > 0], (1, 2)))
    t = out["table"]
    assert abs(t["x"][0] - pos[0][0]) < 0.3 and abs(t["x"][1] - pos[1][0]) \
        < 0.3


def test_faint_companion_below_mincont_stays_merged():
    img, _ = _gauss_pair(5.0, flux=(1e5, 200.0))
    B = np.full_like(img, 100.0)
    R = np.full_like(img, 1.0)
    p = oracle.Params(det_nsigma=5.0)
    det = dt.detect(img, B, R, p)
    out = db.deblend(img, B, R, det["labels"], det["table"], p)
    assert out["n"] == det["n"] == 1


@pytest.mark.parametrize("seed", range(6))
def test_random_blends_partition_their_candidates(seed):
    rng = np.random.default_rng(seed)
    h, w = 48, 64
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    img = 50.0 + rng.normal(0, 1.0, (h, w))
    for _ in range(8):
        xc, yc = rng.uniform(5, w - 5), rng.uniform(5, h - 5)
        f = rng.uniform(50, 3000)
        img += f / (2 * np.pi * 2.0) * np.exp(-((x - xc) ** 2 +
                                                 (y - yc) ** 2) / 4.0)
    img = img.astype(np.float32)
    B = np.full_like(img, 50.0)
    R = np.full_like(img, 1.0)
    p = oracle.Params(det_nsigma=3.0)
    det = dt.detect(img, B, R, p)
    out = db.deblend(img, B, R, det["labels"], det["table"], p)
    o, lab = out["objects"], det["labels"]
    # objects partition the candidates: same support, each object inside
    # one candidate, numbered candidate by candidate
    assert np.array_equal(o > 0, lab > 0)
    par = out["table"]["parent"]
    for k in range(1, out["n"] + 1):
        assert np.all(lab[o == k] == par[k - 1])
    assert np.all(np.diff(par) >= 0)
    assert out["counts"].sum() == out["n"]
    # a candidate with one regional maximum is never split
    v = img.astype(np.float64) - 50.0
    for k in range(1, det["n"] + 1):
        m = lab == k
        peaks = 0
        ys, xs = np.nonzero(m)
        for yy, xx in zip(ys, xs):
            nb = v[max(yy - 1, 0):yy + 2, max(xx - 1, 0):xx + 2]
            mk = m[max(yy - 1, 0):yy + 2, max(xx - 1, 0):xx + 2]
            if v[yy, xx] >= nb[mk].max():
                peaks += 1
        assert out["counts"][k - 1] <= max(peaks, 1)
    # flux is conserved: the objects' fluxes sum to their candidate's
    tc = det["table"]["flux_iso"]
    for k in range(1, det["n"] + 1):
        got = math.fsum(out["table"]["flux_iso"][par == k])
        assert abs(got - tc[k - 1]) <= 1e-9 * abs(tc[k - 1])
