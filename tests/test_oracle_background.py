"""Pins of the background oracle (Sec. 2.2.2) against facts outside it:
hand-worked cases, numpy/scipy routines, closed forms and statistics."""
import math
import os

import numpy as np
import pytest
import scipy.interpolate
import scipy.ndimage
import scipy.stats

from oracle import Params
from oracle import background as bg
from oracle.params import (EST_MEAN, EST_MEDIAN, EST_MODE,
                           FRAME_NO_VALID_MESH, FRAME_EMPTY_MESH)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_median_eq1_hand_and_numpy():
    assert bg.median_eq1([3.0, 1.0, 2.0]) == 2.0
    assert bg.median_eq1([4.0, 1.0, 3.0, 2.0]) == 2.5
    rng = np.random.default_rng(1)
    for n in (1, 2, 7, 64, 4096, 4095):
        v = rng.normal(1000, 30, n).astype(np.float32).astype(np.float64)
        assert bg.median_eq1(v) == float(np.median(v))


def _read_golden_clip():
    """tests/golden/clip_example.txt: values, k, iters, survivors."""
    with open(os.path.join(GOLDEN, "clip_example.txt")) as f:
        rows = [ln.split("#")[0].strip() for ln in f]
    rows = [r for r in rows if r]
    vals = [float(x) for x in rows[0].split()]
    k, iters = float(rows[1].split()[0]), int(rows[1].split()[1])
    surv = [float(x) for x in rows[2].split()]
    stats = [float(x) for x in rows[3].split()]
    return vals, k, iters, surv, stats


def test_clip_golden_example():
    vals, k, iters, surv, (med, mean, var) = _read_golden_clip()
    keep = bg.clip_mask(np.array(vals), iters, k)
    assert sorted(np.array(vals)[keep].tolist()) == surv
    s = np.array(vals)[keep]
    assert bg.median_eq1(s) == med
    assert bg.mean_eq2(s) == mean
    assert bg.std_ddof0(s, bg.mean_eq2(s)) == pytest.approx(math.sqrt(var),
                                                            rel=1e-15)


def test_region_stats_match_numpy_on_survivors():
    rng = np.random.default_rng(2)
    v = rng.normal(800, 25, 4096)
    v[:40] += rng.uniform(1e3, 1e5, 40)               # stars
    v = v.astype(np.float32).astype(np.float64)
    p = Params(estimator=EST_MEAN)
    val, rms, n, med, mean = bg.region_stats(v, p)
    keep = bg.clip_mask(v, p.clip_iters, p.clip_sigma)
    s = v[keep]
    assert n == s.size and n < 4096 - 39
    assert mean == pytest.approx(float(np.mean(s)), rel=1e-15)
    assert rms == pytest.approx(float(np.std(s)), rel=1e-13)
    assert med == float(np.median(s))
    assert val == mean
    assert bg.region_stats(v, Params(estimator=EST_MEDIAN))[0] == med
    assert bg.region_stats(v, Params(estimator=EST_MODE))[0] == \
        3.0 * med - 2.0 * mean
    assert bg.region_stats(v, Params())[0] == 2.5 * med - 1.5 * mean


def test_clip_rejects_only_outliers_and_stops():
    # every survivor lies inside the last bounds, every reject outside one
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(0, 1, 2000), [50.0, -40.0, 30.0]])
    keep = bg.clip_mask(v, 10, 3.0)
    assert not keep[-3:].any()
    s = v[keep]
    c, mu = bg.median_eq1(s), bg.mean_eq2(s)
    sd = bg.std_ddof0(s, mu)
    assert np.all((s >= c - 3 * sd) & (s <= c + 3 * sd))


def test_symmetric_region_gives_centre():
    # values c +- delta, symmetric: median = mean = c, so Eq. 3 gives c
    c = 1234.5
    d = np.arange(1, 2049, dtype=np.float64) * 0.125
    v = np.concatenate([c - d, c + d])
    val, rms, n, med, mean = bg.region_stats(v, Params())
    assert med == c and mean == c and val == c


def test_truncated_normal_recursion():
    # a Gaussian clipped at +-k s_t has std s_{t+1} = g(k s_t) with
    # g(T)^2 = 1 - 2 T phi(T) / (2 Phi(T) - 1)
    rng = np.random.default_rng(4)
    v = rng.normal(0.0, 1.0, 400000)
    def g(T):
        return math.sqrt(1 - 2 * T * scipy.stats.norm.pdf(T)
                         / (2 * scipy.stats.norm.cdf(T) - 1))
    s = 1.0
    for _ in range(3):
        s = g(3.0 * s)
    assert s == pytest.approx(0.98487, abs=2e-5)
    _, rms, _, _, _ = bg.region_stats(v, Params(estimator=EST_MEAN))
    assert rms == pytest.approx(s, rel=4e-3)


def test_mesh_stats_tiling_and_partial_tiles():
    assert bg.tile_bounds(130, 64) == [(0, 64), (64, 128), (128, 130)]
    assert bg.node_centres(130, 64).tolist() == [31.5, 95.5, 128.5]
    img = np.ones((70, 130), dtype=np.float32) * 5
    img[0, 0] = np.nan
    m = np.zeros(img.shape, dtype=bool)
    m[1, 0] = True
    b, r, n, _, _ = bg.mesh_stats(img, Params(min_valid=1), m)
    assert n.tolist() == [[64 * 64 - 2, 64 * 64, 128], [6 * 64, 6 * 64, 12]]
    assert np.all(b == 5.0) and np.all(r == 0.0)


def test_fill_single_hole_and_ring():
    b = np.arange(9, dtype=np.float64).reshape(3, 3) * 10
    n = np.full((3, 3), 200)
    n[1, 1] = 0
    out, _, fl = bg.fill_invalid(b, b, n, 100)
    assert fl == 0
    assert out[1, 1] == (0 + 10 + 20 + 30 + 50 + 60 + 70 + 80) / 8.0
    # 5x5 with a 3x3 hole: ring nodes first, then the centre from the ring
    b = np.arange(25, dtype=np.float64).reshape(5, 5)
    n = np.full((5, 5), 200)
    n[1:4, 1:4] = 0
    out, _, _ = bg.fill_invalid(b, b, n, 100)
    assert out[1, 1] == (0 + 1 + 2 + 5 + 10) / 5.0          # corner of hole
    assert out[1, 2] == (1 + 2 + 3) / 3.0                   # edge of hole
    ring = [out[1, 1], out[1, 2], out[1, 3], out[2, 1], out[2, 3],
            out[3, 1], out[3, 2], out[3, 3]]
    s = 0.0
    for x in ring:
        s += x
    assert out[2, 2] == s / 8.0


def test_fill_fallbacks():
    b = np.full((2, 2), 7.0)
    n = np.array([[5, 0], [0, 0]])
    out, _, fl = bg.fill_invalid(b, b, n, 100)
    assert fl == FRAME_NO_VALID_MESH and np.all(out == 7.0)
    out, outr, fl = bg.fill_invalid(b, b, np.zeros((2, 2), int), 100)
    assert fl == FRAME_NO_VALID_MESH | FRAME_EMPTY_MESH
    assert np.all(out == 0) and np.all(outr == 0)


def test_median_filter_interior_matches_scipy_and_edges_shrink():
    rng = np.random.default_rng(5)
    m = rng.normal(size=(9, 11))
    out = bg.median_filter(m, 3, 3)
    ref = scipy.ndimage.median_filter(m, size=3, mode="nearest")
    assert np.array_equal(out[1:-1, 1:-1], ref[1:-1, 1:-1])
    # corner window is 2x2: mean of the two middle values
    s = np.sort(m[:2, :2].ravel())
    assert out[0, 0] == (s[1] + s[2]) / 2.0
    assert np.array_equal(bg.median_filter(m, 1, 1), m)
    # a plane: interior kept, edge node moves to its window centre
    plane = np.tile(np.arange(5, dtype=np.float64) * 32, (4, 1))
    f = bg.median_filter(plane, 3, 3)
    assert np.array_equal(f[:, 1:-1], plane[:, 1:-1])
    assert np.all(f[:, 0] == 16.0)


def test_spline_matches_scipy_natural_inside_and_linear_outside():
    rng = np.random.default_rng(6)
    t = np.cumsum(rng.uniform(20, 70, 9))
    f = rng.normal(1000, 30, 9)
    M = bg.natural_second_derivatives(t, f)
    cs = scipy.interpolate.CubicSpline(t, f, bc_type="natural")
    xq = np.linspace(t[0], t[-1], 333)
    assert np.allclose(bg.spline_eval(t, f, M, xq), cs(xq), rtol=0,
                       atol=1e-10)
    assert np.allclose(M, cs(t, 2), atol=1e-10)
    d1 = cs.derivative()
    xl = t[0] - np.array([0.5, 7.0, 31.5])
    xr = t[-1] + np.array([0.5, 7.0, 31.5])
    assert np.allclose(bg.spline_eval(t, f, M, xl),
                       cs(t[0]) + d1(t[0]) * (xl - t[0]), atol=1e-10)
    assert np.allclose(bg.spline_eval(t, f, M, xr),
                       cs(t[-1]) + d1(t[-1]) * (xr - t[-1]), atol=1e-10)


def test_spline_degenerate_node_counts():
    one = bg.spline_eval(np.array([3.0]), np.array([5.0]), np.zeros(1),
                         np.arange(7.0))
    assert np.all(one == 5.0)
    t = np.array([31.5, 95.5])
    f = np.array([10.0, 42.0])
    y = bg.spline_eval(t, f, bg.natural_second_derivatives(t, f),
                       np.arange(128.0))
    assert np.allclose(y, 10.0 + 0.5 * (np.arange(128.0) - 31.5), atol=1e-12)


def test_interpolate_nodes_and_bilinear_exact():
    p = Params(mesh_h=16, mesh_w=32)
    h, w = 70, 150                                        # ragged tiles
    yc, xc = bg.node_centres(h, 16), bg.node_centres(w, 32)
    rng = np.random.default_rng(7)
    mesh = rng.normal(500, 20, (yc.size, xc.size))
    out = bg.interpolate(mesh, h, w, p)
    for j, y in enumerate(yc):
        for i, x in enumerate(xc):
            if float(y).is_integer() and float(x).is_integer():
                assert out[int(y), int(x)] == pytest.approx(mesh[j, i],
                                                            abs=1e-9)
    a, b, c, d = 700.0, 0.25, -0.75, 1e-3
    lin = a + b * xc[None, :] + c * yc[:, None] + d * xc[None, :] * yc[:, None]
    out = bg.interpolate(lin, h, w, p)
    X, Y = np.meshgrid(np.arange(w), np.arange(h))
    assert np.allclose(out, a + b * X + c * Y + d * X * Y, rtol=0, atol=1e-9)


def test_noise_free_plane_frame_gives_the_plane():
    h, w = 200, 300
    img = (1000.0 + 0.5 * np.arange(w))[None, :].repeat(h, 0)
    img = img.astype(np.float32)
    p = Params(filter_h=1, filter_w=1)
    out = bg.background(img, p)
    assert out["flags"] == 0
    X = np.arange(w)[None, :].repeat(h, 0)
    assert np.allclose(out["B64"], 1000.0 + 0.5 * X, rtol=0, atol=1e-9)
    assert np.array_equal(out["B32"], img)
