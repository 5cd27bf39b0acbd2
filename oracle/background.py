"""Background estimation and removal, Sec. 2.2.2 of the paper, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order:

1. segment the frame into rectangular regions (default 64x64 px);
2. in each region, iterate: estimate a central value and a standard
   deviation, reject the pixels outside centre +- k sigma, until the iteration
   limit is reached or nothing more is rejected (the data stabilise);
3. turn the surviving pixels into one value per region with one of the four
   estimators of Eq. 1-4;
4. smooth the mesh of region values with a median filter;
5. interpolate the mesh back to the full image resolution with a spline.

Readings taken where the text is open (each is a choice, not the paper's):

* Partial regions at the right/bottom edge are kept; a node sits at the
  centre of its region's actual pixel extent.
* The clip centre is the median (Eq. 1), the scale the population (ddof 0)
  standard deviation, the bounds are inclusive, at most ``clip_iters``
  rejection passes are made, and the final statistics are those of the
  survivors.  Mean and variance sums are exact (``math.fsum``) and rounded
  once; the deviations (v - mean)^2 are binary64 products.
* Eq. 3 is the "2.5 median - 1.5 mean" estimator (the paper calls it the
  sigma estimator); it is the default and has no fallback.  Eq. 4 is printed
  with the mean twice; it is read as median_factor*median - mean_factor*mean.
* A region is valid when at least ``min_valid`` pixels survive (the paper's
  "at least 100 pixels").  Invalid nodes are filled by Jacobi passes: each
  pass gives every still-unknown node with at least one known 8-neighbour the
  mean of those neighbours (summed in raster order), until none is unknown.
  If no node is valid, every node with at least one pixel is used; if none
  has a pixel, the background and rms are 0.
* The median filter window shrinks at the mesh edges; even counts use Eq. 1.
* The spline is a tensor-product natural cubic spline through the node
  centres, extended linearly with the end slope outside the first/last node;
  one node gives a constant, two nodes a straight line.
* The maps handed to detection are the binary32 roundings of the binary64
  background and rms.
"""
from __future__ import annotations

import math

import numpy as np

from .params import (Params, EST_SEXTRACTOR, EST_MEDIAN, EST_MEAN, EST_MODE,
                     FRAME_NO_VALID_MESH, FRAME_EMPTY_MESH)


# --------------------------------------------------------------------------
# Step 1: tiling
# --------------------------------------------------------------------------
def tile_bounds(n: int, m: int):
    """[start, stop) of each region along an axis of n pixels, size m."""
    return [(s, min(s + m, n)) for s in range(0, n, m)]


def node_centres(n: int, m: int) -> np.ndarray:
    """Pixel coordinate of each region centre along one axis."""
    return np.array([(a + b - 1) / 2.0 for a, b in tile_bounds(n, m)],
                    dtype=np.float64)


# --------------------------------------------------------------------------
# Steps 2-3: clipped statistics and the estimators (Eq. 1-4)
# --------------------------------------------------------------------------
def median_eq1(values) -> float:
    """Eq. 1: the middle order statistic, or the mean of the two middle ones."""
    s = np.sort(np.asarray(values, dtype=np.float64))
    n = s.size
    if n == 0:
        return math.nan
    if n % 2 == 1:
        return float(s[(n - 1) // 2])
    return (float(s[n // 2 - 1]) + float(s[n // 2])) / 2.0


def mean_eq2(values) -> float:
    """Eq. 2: arithmetic mean; the sum is exact and rounded once."""
    n = len(values)
    return math.fsum(values) / n if n else math.nan


def std_ddof0(values, mu: float) -> float:
    """Population standard deviation about ``mu``."""
    n = len(values)
    if n == 0:
        return math.nan
    return math.sqrt(math.fsum((float(v) - mu) * (float(v) - mu)
                               for v in values) / n)


def clip_mask(values: np.ndarray, iters: int, k: float) -> np.ndarray:
    """Iterative k-sigma clipping about the median; returns the survivor mask.

    Each pass computes the median c, the mean and the population standard
    deviation s of the current members, keeps those with c - k*s <= v <=
    c + k*s, and stops early once a pass rejects nothing.
    """
    v = np.asarray(values, dtype=np.float64)
    keep = np.ones(v.size, dtype=bool)
    for _ in range(iters):
        cur = v[keep]
        if cur.size == 0:
            break
        c = median_eq1(cur)
        mu = mean_eq2(cur)
        s = std_ddof0(cur, mu)
        lo = c - k * s
        hi = c + k * s
        new = keep & (v >= lo) & (v <= hi)
        if new.sum() == keep.sum():
            break
        keep = new
    return keep


def estimator_value(med: float, mean: float, p: Params) -> float:
    if p.estimator == EST_SEXTRACTOR:
        return 2.5 * med - 1.5 * mean                      # Eq. 3
    if p.estimator == EST_MEDIAN:
        return med                                         # Eq. 1
    if p.estimator == EST_MEAN:
        return mean                                        # Eq. 2
    if p.estimator == EST_MODE:
        return p.median_factor * med - p.mean_factor * mean  # Eq. 4
    raise ValueError(p.estimator)


def region_stats(values: np.ndarray, p: Params):
    """Clipped statistics of one region: (value, rms, n_used, median, mean)."""
    v = np.asarray(values, dtype=np.float64)
    keep = clip_mask(v, p.clip_iters, p.clip_sigma)
    s = v[keep]
    if s.size == 0:
        return math.nan, math.nan, 0, math.nan, math.nan
    med = median_eq1(s)
    mu = mean_eq2(s)
    sd = std_ddof0(s, mu)
    return estimator_value(med, mu, p), sd, int(s.size), med, mu


def mesh_stats(frame: np.ndarray, p: Params, mask: np.ndarray | None = None):
    """Per-region value, rms and survivor count; non-finite or masked pixels
    (mask true) are not used."""
    img = np.asarray(frame)
    h, w = img.shape
    rows, cols = tile_bounds(h, p.mesh_h), tile_bounds(w, p.mesh_w)
    bkg = np.full((len(rows), len(cols)), math.nan)
    rms = np.full_like(bkg, math.nan)
    med = np.full_like(bkg, math.nan)
    mean = np.full_like(bkg, math.nan)
    n = np.zeros(bkg.shape, dtype=np.int64)
    for j, (y0, y1) in enumerate(rows):
        for i, (x0, x1) in enumerate(cols):
            t = img[y0:y1, x0:x1].astype(np.float64).ravel()
            ok = np.isfinite(t)
            if mask is not None:
                ok &= ~np.asarray(mask[y0:y1, x0:x1], dtype=bool).ravel()
            b, r, c, md, mu = region_stats(t[ok], p)
            bkg[j, i], rms[j, i], n[j, i] = b, r, c
            med[j, i], mean[j, i] = md, mu
    return bkg, rms, n, med, mean


# --------------------------------------------------------------------------
# Invalid-node fill
# --------------------------------------------------------------------------
def fill_invalid(bkg: np.ndarray, rms: np.ndarray, n: np.ndarray,
                 min_valid: int):
    """Replace the values of invalid nodes; returns (bkg, rms, frame_flags)."""
    flags = 0
    known = n >= min_valid
    if not known.any():
        flags |= FRAME_NO_VALID_MESH
        known = n >= 1
    if not known.any():
        flags |= FRAME_EMPTY_MESH
        return np.zeros_like(bkg), np.zeros_like(rms), flags
    b = np.where(known, bkg, 0.0).astype(np.float64)
    r = np.where(known, rms, 0.0).astype(np.float64)
    ny, nx = b.shape
    while not known.all():
        upd = []
        for j in range(ny):
            for i in range(nx):
                if known[j, i]:
                    continue
                sb = 0.0
                sr = 0.0
                cnt = 0
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        jj, ii = j + dj, i + di
                        if (dj or di) and 0 <= jj < ny and 0 <= ii < nx \
                                and known[jj, ii]:
                            sb += b[jj, ii]
                            sr += r[jj, ii]
                            cnt += 1
                if cnt:
                    upd.append((j, i, sb / cnt, sr / cnt))
        for j, i, vb, vr in upd:
            b[j, i], r[j, i] = vb, vr
            known[j, i] = True
    return b, r, flags


# --------------------------------------------------------------------------
# Step 4: median filter of the mesh
# --------------------------------------------------------------------------
def median_filter(mesh: np.ndarray, fh: int, fw: int) -> np.ndarray:
    ny, nx = mesh.shape
    out = np.empty_like(mesh)
    for j in range(ny):
        for i in range(nx):
            win = mesh[max(0, j - fh // 2):min(ny, j + fh // 2 + 1),
                       max(0, i - fw // 2):min(nx, i + fw // 2 + 1)]
            out[j, i] = median_eq1(win.ravel())
    return out


# --------------------------------------------------------------------------
# Step 5: natural cubic spline interpolation back to full resolution
# --------------------------------------------------------------------------
def natural_second_derivatives(t: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Second derivatives of the natural cubic spline through (t, f).

    ``f`` may carry trailing dimensions (several splines on the same knots).
    Interior equations: h[i-1] M[i-1] + 2 (h[i-1] + h[i]) M[i] + h[i] M[i+1]
    = 6 ((f[i+1]-f[i])/h[i] - (f[i]-f[i-1])/h[i-1]); M = 0 at both ends.
    Solved densely (slow but plain).
    """
    t = np.asarray(t, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    n = t.size
    M = np.zeros_like(f)
    if n < 3:
        return M
    h = np.diff(t)
    A = np.zeros((n - 2, n - 2))
    rhs = np.zeros((n - 2,) + f.shape[1:])
    for i in range(1, n - 1):
        r = i - 1
        if r > 0:
            A[r, r - 1] = h[i - 1]
        A[r, r] = 2.0 * (h[i - 1] + h[i])
        if r < n - 3:
            A[r, r + 1] = h[i]
        rhs[r] = 6.0 * ((f[i + 1] - f[i]) / h[i] - (f[i] - f[i - 1]) / h[i - 1])
    M[1:-1] = np.linalg.solve(A, rhs)
    return M


def spline_eval(t: np.ndarray, f: np.ndarray, M: np.ndarray,
                xq: np.ndarray) -> np.ndarray:
    """Evaluate the spline (t, f, M) at ``xq``; linear beyond the end knots
    with the end slope.  Returns shape (len(xq),) + f.shape[1:]."""
    t = np.asarray(t, dtype=np.float64)
    xq = np.asarray(xq, dtype=np.float64)
    n = t.size
    ext = (slice(None),) + (None,) * (f.ndim - 1)
    if n == 1:
        return np.broadcast_to(f[0], (xq.size,) + f.shape[1:]).copy()
    i = np.clip(np.searchsorted(t, xq, side="right") - 1, 0, n - 2)
    h = (t[i + 1] - t[i])[ext]
    a = ((t[i + 1] - xq)[ext]) / h
    b = ((xq - t[i])[ext]) / h
    inner = (a * f[i] + b * f[i + 1]
             + ((a * a * a - a) * M[i] + (b * b * b - b) * M[i + 1])
             * (h * h) / 6.0)
    h0 = t[1] - t[0]
    s0 = (f[1] - f[0]) / h0 - h0 * (2.0 * M[0] + M[1]) / 6.0
    hn = t[-1] - t[-2]
    sn = (f[-1] - f[-2]) / hn + hn * (M[-2] + 2.0 * M[-1]) / 6.0
    left = f[0] + s0 * ((xq - t[0])[ext])
    right = f[-1] + sn * ((xq - t[-1])[ext])
    below = (xq < t[0])[ext]
    above = (xq > t[-1])[ext]
    return np.where(below, left, np.where(above, right, inner))


def interpolate(mesh: np.ndarray, h: int, w: int, p: Params) -> np.ndarray:
    """Full-resolution map from a mesh: spline along y for every mesh column,
    then along x for every image row."""
    yc = node_centres(h, p.mesh_h)
    xc = node_centres(w, p.mesh_w)
    My = natural_second_derivatives(yc, mesh)                  # (ny, nx)
    G = spline_eval(yc, mesh, My, np.arange(h))                # (h, nx)
    Mx = natural_second_derivatives(xc, G.T)                   # (nx, h)
    return spline_eval(xc, G.T, Mx, np.arange(w)).T.copy()     # (h, w)


# --------------------------------------------------------------------------
# The whole step
# --------------------------------------------------------------------------
def background(frame: np.ndarray, p: Params, mask: np.ndarray | None = None):
    """Background and rms maps of one frame, with the intermediate meshes."""
    img = np.asarray(frame, dtype=np.float32)
    h, w = img.shape
    bkg_raw, rms_raw, n, med, mean = mesh_stats(img, p, mask)
    bkg_f, rms_f, flags = fill_invalid(bkg_raw, rms_raw, n, p.min_valid)
    bkg_m = median_filter(bkg_f, p.filter_h, p.filter_w)
    rms_m = median_filter(rms_f, p.filter_h, p.filter_w)
    B64 = interpolate(bkg_m, h, w, p)
    R64 = interpolate(rms_m, h, w, p)
    return {
        "bkg_raw": bkg_raw, "rms_raw": rms_raw, "n_used": n,
        "median": med, "mean": mean,
        "bkg_filled": bkg_f, "rms_filled": rms_f,
        "bkg_mesh": bkg_m, "rms_mesh": rms_m,
        "B64": B64, "R64": R64,
        "B32": B64.astype(np.float32), "R32": R64.astype(np.float32),
        "flags": flags,
    }
