"""Source detection and pre-analysis, Sec. 2.2.5 of the paper, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order: every pixel whose background-subtracted value
exceeds the main threshold is detected; detected pixels are connected into
candidates; each candidate's peak value and total flux are measured
(pre-analysis).  Deblending and cleaning are not part of this path.

Readings taken where the text is open:

* v = (double)I - (double)B32 with B32 the binary32 background map; the
  threshold is t = nsigma * (double)R32 with R32 the binary32 rms map; a pixel
  is detected iff I is finite and v > t (strict).  No detection filter.
* Candidates are 8-connected (4-connected on request) sets of detected
  pixels; those with fewer than ``min_area`` pixels are dropped.  Labels are
  1..K in increasing order of each candidate's first pixel in raster order
  (row-major), 0 elsewhere.
* Pre-analysis per candidate: pixel count, bounding box, peak value (ties go
  to the lowest raster index), isophotal flux S = sum v and the
  flux-weighted barycentre xmin + Sx/S, ymin + Sy/S with Sx = sum v (x-xmin).
  Sums are exact: each v is taken as the integer D = round(v * 2^28) (exact
  when I and B32 are 0 or of magnitude in [2^-5, 2^24]; otherwise the row is
  flagged), summed as integers and rounded once to binary64.  The
  barycentre is fl(xmin + fl(fl(Sx) / fl(S))).  When S <= 0 the unweighted
  pixel mean is used instead and the row is flagged.
"""
from __future__ import annotations

import math

import numpy as np

from .params import (Params, SRC_INEXACT_SUM_RANGE, SRC_NONPOSITIVE_FLUX)

_Q = 28                       # fixed-point fraction bits of the exact sums
_DMAX = (1 << 62) - 1         # |D| clamp


def threshold(frame: np.ndarray, B32: np.ndarray, R32: np.ndarray,
              nsigma: float):
    """Detection mask and the subtracted values v (binary64)."""
    I = np.asarray(frame, dtype=np.float32).astype(np.float64)
    v = I - np.asarray(B32, dtype=np.float32).astype(np.float64)
    t = nsigma * np.asarray(R32, dtype=np.float32).astype(np.float64)
    det = np.isfinite(I) & (v > t)
    return det, v


def _neighbours(connectivity: int):
    if connectivity == 8:
        return [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0),
                (1, 1)]
    if connectivity == 4:
        return [(-1, 0), (0, -1), (0, 1), (1, 0)]
    raise ValueError(connectivity)


def label_components(det: np.ndarray, connectivity: int = 8):
    """Flood fill started from each unlabelled detected pixel in raster
    order; returns (labels int32, count)."""
    h, w = det.shape
    lab = np.zeros((h, w), dtype=np.int32)
    nb = _neighbours(connectivity)
    n = 0
    ys, xs = np.nonzero(det)                       # raster order
    for y0, x0 in zip(ys.tolist(), xs.tolist()):
        if lab[y0, x0]:
            continue
        n += 1
        lab[y0, x0] = n
        stack = [(y0, x0)]
        while stack:
            y, x = stack.pop()
            for dy, dx in nb:
                yy, xx = y + dy, x + dx
                if 0 <= yy < h and 0 <= xx < w and det[yy, xx] \
                        and not lab[yy, xx]:
                    lab[yy, xx] = n
                    stack.append((yy, xx))
    return lab, n


def apply_min_area(lab: np.ndarray, n: int, min_area: int):
    """Drop candidates below ``min_area`` pixels and renumber the rest in
    their original order."""
    sizes = np.bincount(lab.ravel(), minlength=n + 1)
    keep = sizes >= min_area
    keep[0] = False
    new = np.zeros(n + 1, dtype=np.int32)
    new[keep] = np.arange(1, int(keep.sum()) + 1, dtype=np.int32)
    return new[lab], int(keep.sum())


def _exact_range(a: float) -> bool:
    a = abs(a)
    return a == 0.0 or (2.0 ** -5 <= a <= 2.0 ** 24)


def source_table(frame: np.ndarray, B32: np.ndarray, lab: np.ndarray,
                 nlab: int):
    """Pre-analysis of every labelled candidate (dict of arrays, row k is
    label k+1)."""
    I32 = np.asarray(frame, dtype=np.float32)
    B = np.asarray(B32, dtype=np.float32)
    h, w = lab.shape
    flat = lab.ravel()
    order = np.argsort(flat, kind="stable")        # raster order per label
    starts = np.searchsorted(flat[order], np.arange(nlab + 2))
    cols = {k: [] for k in ("label", "npix", "xmin", "xmax", "ymin", "ymax",
                            "peak", "peak_x", "peak_y", "flux_iso", "x", "y",
                            "flags")}
    for k in range(1, nlab + 1):
        idx = order[starts[k]:starts[k + 1]]
        ys, xs = idx // w, idx % w
        Iv = I32.ravel()[idx]
        Bv = B.ravel()[idx]
        v = Iv.astype(np.float64) - Bv.astype(np.float64)
        xmin, xmax = int(xs.min()), int(xs.max())
        ymin, ymax = int(ys.min()), int(ys.max())
        j = int(np.argmax(v))                      # first max = lowest index
        flags = 0
        S = Sx = Sy = 0
        for vi, xi, yi, a, b in zip(v.tolist(), xs.tolist(), ys.tolist(),
                                    Iv.tolist(), Bv.tolist()):
            D = int(round(vi * 2.0 ** _Q))
            if not (_exact_range(a) and _exact_range(b)):
                flags |= SRC_INEXACT_SUM_RANGE
            if D > _DMAX or D < -_DMAX:
                D = _DMAX if D > 0 else -_DMAX
                flags |= SRC_INEXACT_SUM_RANGE
            S += D
            Sx += D * (xi - xmin)
            Sy += D * (yi - ymin)
        if S > 0:
            fS = float(S)
            cx = xmin + float(Sx) / fS
            cy = ymin + float(Sy) / fS
        else:
            flags |= SRC_NONPOSITIVE_FLUX
            cx = xmin + float(int(np.sum(xs - xmin))) / float(xs.size)
            cy = ymin + float(int(np.sum(ys - ymin))) / float(ys.size)
        cols["label"].append(k)
        cols["npix"].append(int(idx.size))
        cols["xmin"].append(xmin)
        cols["xmax"].append(xmax)
        cols["ymin"].append(ymin)
        cols["ymax"].append(ymax)
        cols["peak"].append(float(v[j]))
        cols["peak_x"].append(int(xs[j]))
        cols["peak_y"].append(int(ys[j]))
        cols["flux_iso"].append(float(S) * 2.0 ** -_Q)
        cols["x"].append(cx)
        cols["y"].append(cy)
        cols["flags"].append(flags)
    out = {}
    for key, vals in cols.items():
        dt = np.float64 if key in ("peak", "flux_iso", "x", "y") else np.int64
        out[key] = np.asarray(vals, dtype=dt)
    return out


def detect(frame: np.ndarray, B32: np.ndarray, R32: np.ndarray, p: Params):
    """Threshold, connect, drop small candidates, pre-analyse."""
    det, _ = threshold(frame, B32, R32, p.det_nsigma)
    lab, n = label_components(det, p.connectivity)
    lab, n = apply_min_area(lab, n, p.min_area)
    return {"det": det, "labels": lab, "n": n,
            "table": source_table(frame, B32, lab, n)}


def source_moments(frame: np.ndarray, B32: np.ndarray, lab: np.ndarray,
                   nlab: int):
    """Second-order moments of every candidate's footprint and the ellipse
    they describe (the pre-analysis of Sec. 2.2.5 carried to second order,
    as SExtractor's X2, Y2, XY, A, B, THETA).  Weights D_i are the same
    integers as in ``source_table`` (d_i 2^28, clipped likewise); with
    dx = x - xmin and dy = y - ymin the exact sums S = sum D, Sx = sum D dx,
    Sy, Sxx = sum D dx^2, Syy, Sxy = sum D dx dy are each rounded to binary64
    once, and then (binary64, in this order):
      mx = Sx / S, my = Sy / S,
      x2 = Sxx / S - mx mx, y2 = Syy / S - my my, xy = Sxy / S - mx my,
      t = (x2 + y2) / 2, h = (x2 - y2) / 2, r = sqrt(h h + xy xy),
      a = sqrt(t + r), b = sqrt(max(t - r, 0)),
      theta = atan2(2 xy, x2 - y2) / 2.
    Returns float64 [nlab, 6] (x2, y2, xy, a, b, theta); NaN where S <= 0.
    """
    I32 = np.asarray(frame, dtype=np.float32)
    B = np.asarray(B32, dtype=np.float32)
    h, w = lab.shape
    flat = lab.ravel()
    order = np.argsort(flat, kind="stable")
    starts = np.searchsorted(flat[order], np.arange(nlab + 2))
    out = np.full((nlab, 6), np.nan)
    for k in range(1, nlab + 1):
        idx = order[starts[k]:starts[k + 1]]
        ys, xs = idx // w, idx % w
        v = (I32.ravel()[idx].astype(np.float64)
             - B.ravel()[idx].astype(np.float64))
        xmin, ymin = int(xs.min()), int(ys.min())
        S = Sx = Sy = Sxx = Syy = Sxy = 0
        for vi, xi, yi in zip(v.tolist(), xs.tolist(), ys.tolist()):
            D = int(round(vi * 2.0 ** _Q))
            if D > _DMAX or D < -_DMAX:
                D = _DMAX if D > 0 else -_DMAX
            dx, dy = xi - xmin, yi - ymin
            S += D
            Sx += D * dx
            Sy += D * dy
            Sxx += D * dx * dx
            Syy += D * dy * dy
            Sxy += D * dx * dy
        if S <= 0:
            continue
        fS = float(S)
        mx = float(Sx) / fS
        my = float(Sy) / fS
        x2 = float(Sxx) / fS - mx * mx
        y2 = float(Syy) / fS - my * my
        xy = float(Sxy) / fS - mx * my
        t = (x2 + y2) / 2.0
        hd = (x2 - y2) / 2.0
        r = math.sqrt(hd * hd + xy * xy)
        a = math.sqrt(t + r)
        b = math.sqrt(max(t - r, 0.0))
        theta = math.atan2(2.0 * xy, x2 - y2) / 2.0
        out[k - 1] = (x2, y2, xy, a, b, theta)
    return out

