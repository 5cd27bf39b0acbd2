"""Pins of the gray-scale oracle (Sec. 2.2.6): zscale, point maps and
histogram equalization against closed forms, hand-worked cases and numpy's
histogram routine."""
import math

import numpy as np
import pytest

from oracle import gray


# ------------------------------------------------------------------ zscale
@pytest.mark.parametrize("h,w,s,n", [
    (4096, 4096, 133, 961),      # 4096/132 -> 32 x 32 = 1024 > 1000
    (2048, 2048, 67, 961),
    (20, 30, 1, 600),
    (1, 32767, 33, 993),
    (10560, 10560, 341, 961),
])
def test_sample_stride(h, w, s, n):
    assert gray.sample_stride(h, w) == s
    assert -(-h // s) * -(-w // s) == n
    assert -(-h // (s - 1)) * -(-w // (s - 1)) > 1000 if s > 1 else True


def test_sample_skips_nonfinite():
    f = np.arange(20 * 25, dtype=np.float32).reshape(20, 25)
    f[3, 4] = np.nan
    f[7, 0] = np.inf
    v = gray.zscale_sample(f)
    assert v.size == 498 and np.all(np.diff(v) >= 0)


def _ramp(n, a=7, b=3, extra=()):
    vals = [a + b * i for i in range(n)] + list(extra)
    rng = np.random.default_rng(4)
    return rng.permutation(np.array(vals, dtype=np.float32))[None, :]


def test_exact_ramp_closed_form():
    # 500 samples 7 + 3 i: the line fits exactly, nothing is rejected;
    # median (even n) = 7 + 3 * 249.5 = 755.5, centre index 249
    f = _ramp(500).reshape(20, 25)
    z1, z2, info = gray.zscale(f, contrast=1.0)
    assert info["slope"] == 3.0 and info["kept"] == 500
    assert info["fits"] == 1 and info["median"] == 755.5
    assert (z1, z2) == (755.5 - 249 * 3, 1504.0)        # 8.5, clamped top
    z1, z2, _ = gray.zscale(f, contrast=2.0)
    assert (z1, z2) == (755.5 - 249 * 1.5, 755.5 + 250 * 1.5)
    z1, z2, _ = gray.zscale(f)                          # contrast 0.25
    assert (z1, z2) == (7.0, 1504.0)                    # both clamped


def test_outliers_rejected_with_growth():
    # 500 ramp samples and 3 outliers on top (n = 503, odd): the first fit
    # rejects the outliers and, grown by ngrow // 2 = 2, samples 498, 499;
    # the second fit is exact (slope 3) and rejects nothing new, which
    # ends the iteration
    f = _ramp(500, extra=(1e6, 2e6, 3e6))
    z1, z2, info = gray.zscale(f, contrast=1.0)
    assert info["n"] == 503 and info["kept"] == 498
    assert info["slope"] == 3.0 and info["fits"] == 2
    med = 7 + 3 * 251
    assert info["median"] == med
    assert (z1, z2) == (7.0, med + 251 * 3)


def test_too_few_samples_fall_back_to_extremes():
    f = np.array([[5.0, -2.0, 9.0, 4.0]], dtype=np.float32)
    z1, z2, info = gray.zscale(f)
    assert (z1, z2) == (-2.0, 9.0) and info["fits"] == 0
    z1, z2, info = gray.zscale(np.full((3, 3), np.nan, dtype=np.float32))
    assert (z1, z2, info["n"]) == (0.0, 0.0, 0)


def test_noise_range_brackets_the_median():
    rng = np.random.default_rng(9)
    f = rng.normal(1000.0, 30.0, (512, 512)).astype(np.float32)
    z1, z2, info = gray.zscale(f)
    assert z1 < info["median"] < z2
    # for Gaussian data the sorted sample's central slope is about
    # sigma sqrt(2 pi) / n, so the range is about sqrt(2 pi) sigma / 0.25
    assert 0.6 < (z2 - z1) / (math.sqrt(2 * math.pi) * 30 / 0.25) < 1.4


# -------------------------------------------------------------- point maps
@pytest.mark.parametrize("kind", [gray.LINEAR, gray.LOG, gray.EXP,
                                  gray.POWER])
def test_maps_fix_the_ends_and_are_monotone(kind):
    a = 0.5 if kind == gray.POWER else 1000.0
    v = np.linspace(-50.0, 150.0, 401)
    y = gray.point_map(v, kind, 0.0, 100.0, a)
    assert y[v <= 0].max() == 0.0
    assert np.all(np.abs(y[v >= 100] - 1.0) <= 1e-15)
    assert np.all(np.diff(y) >= 0)


def test_map_closed_forms():
    lo, hi = 10.0, 30.0
    mid = np.array([20.0])
    assert gray.point_map(mid, gray.LINEAR, lo, hi)[0] == 0.5
    # exponential at x = 1/2: (sqrt(a) - 1) / (a - 1) = 1 / (sqrt(a) + 1)
    a = 400.0
    assert math.isclose(gray.point_map(mid, gray.EXP, lo, hi, a)[0],
                        1.0 / 21.0, rel_tol=1e-15)
    # power law x^(1/2) at x = 1/4
    assert gray.point_map(np.array([15.0]), gray.POWER, lo, hi, 0.5)[0] == 0.5
    # logarithmic at x = 1/2 with a = 2: ln 2 / ln 3
    assert math.isclose(gray.point_map(mid, gray.LOG, lo, hi, 2.0)[0],
                        math.log(2) / math.log(3), rel_tol=1e-15)
    # NaN stays NaN; a degenerate range is a step at lo
    assert np.isnan(gray.point_map(np.array([np.nan]), gray.LINEAR, lo, hi)[0])
    s = gray.point_map(np.array([9.0, 10.0, 11.0]), gray.LINEAR, 10.0, 10.0)
    assert s.tolist() == [0.0, 0.0, 1.0]


# -------------------------------------------------- histogram equalization
def test_two_levels_closed_form():
    m, n = 700, 1000
    f = np.zeros(n, dtype=np.float32)
    f[m:] = 1.0
    for nb in (2, 4096):
        y, counts, lo, hi = gray.equalize_hist(f[None, :], nb)
        assert counts[0] == m and counts[-1] == n - m
        assert np.all(y[0, :m] == m / n) and np.all(y[0, m:] == 1.0)


def test_three_levels_interpolated():
    # values 0, 1/2, 1 with counts a, b, c and two bins: cdf = [a/N, 1] at
    # centres 1/4, 3/4, so the middle level maps to (a/N + 1) / 2
    a, b, c = 300, 500, 200
    f = np.array([0.0] * a + [0.5] * b + [1.0] * c, dtype=np.float32)
    y, counts, _, _ = gray.equalize_hist(f[None, :], 2)
    assert counts.tolist() == [a, b + c]
    assert np.allclose(y[0, a:a + b], (a / 1000 + 1.0) / 2, rtol=1e-15,
                       atol=0)


def test_counts_match_numpy_histogram():
    rng = np.random.default_rng(3)
    f = rng.integers(0, 1000, (64, 64)).astype(np.float32)
    f[0, 0], f[0, 1] = 0.0, 999.0
    _, counts, lo, hi = gray.equalize_hist(f, 1000)
    ref, _ = np.histogram(f, bins=1000, range=(0.0, 999.0))
    assert (lo, hi) == (0.0, 999.0)
    assert np.array_equal(counts, ref)


def test_constant_and_nonfinite():
    f = np.full((8, 8), 3.5, dtype=np.float32)
    f[1, 1] = np.nan
    y, counts, _, _ = gray.equalize_hist(f)
    assert np.isnan(y[1, 1]) and np.all(y[np.isfinite(f)] == 1.0)
    assert counts[0] == 63


def test_uniform_data_is_nearly_identity():
    rng = np.random.default_rng(8)
    f = rng.uniform(100.0, 200.0, (256, 256)).astype(np.float32)
    y, _, lo, hi = gray.equalize_hist(f)
    x = (f.astype(np.float64) - lo) / (hi - lo)
    assert np.max(np.abs(y - x)) < 3.0 / 256 + 2.0 / 4096
    order = np.argsort(f.ravel(), kind="stable")
    assert np.all(np.diff(y.ravel()[order]) >= 0)
