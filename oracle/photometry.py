"""Aperture photometry with a local sky annulus, and its adjoint, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2.5 of the paper measures each object's flux in a circular aperture,
one object per GPU thread; the aperture geometry and the sky are not spelled
out.  Readings taken here:

* Pixel (x, y) covers [x-1/2, x+1/2] x [y-1/2, y+1/2].  The aperture weight of
  a pixel is the exact area of its intersection with the disk of radius
  r_ap about the centroid; the annulus weight is the same area for r_out
  minus that for r_in.
* The area comes from the signed corner integral
  G(x, y) = int_0^x int_0^y [s^2 + t^2 <= r^2] dt ds (odd in x and in y), by
  inclusion-exclusion over the four pixel corners.  For 0 <= x, y <= r:
  G = x*y when the corner is inside the circle, else
  G = y*xs + P(x) - P(xs) with xs = sqrt(r^2 - y^2) and
  P(s) = int_0^s sqrt(r^2 - u^2) du = (s sqrt(r^2 - s^2) + r^2 asin(s/r))/2.
* A pixel belongs to an aperture (disk of radius r) iff its square meets the
  open disk: with dx = max(|x - cx| - 1/2, 0) and dy likewise,
  dx^2 + dy^2 < r^2.  It lies wholly inside iff (|x-cx|+1/2)^2 +
  (|y-cy|+1/2)^2 <= r^2; its weight is then 1, for non-members 0, and
  otherwise the exact area below.  A pixel belongs to the annulus iff it
  meets the disk of radius r_out and is not wholly inside the disk of
  radius r_in.  Membership is decided by these predicates (evaluated in
  binary64 in exactly this form), not by the sign of a computed area, so
  that a rounding residue never adds a pixel to the sky sample.
* Only member pixels inside the frame with a finite value count; a member
  pixel outside the frame or not finite flags the source.
* Values are v = (double)I - (double)B32.  The sky is the weighted mean
  sum(m w v) / sum(m w) over annulus pixels, with m the survivors of the same
  k-sigma clipping as the background regions (median centre, population
  sigma, inclusive bounds, at most ``sky_clip_iters`` passes) applied to the
  unweighted annulus values.  Flux = sum(w_ap v) - sky * sum(w_ap).
* Adjoint (sky mask m held fixed):
  dF/dv_i = w_ap_i - A_ap m_i w_ann_i / A_ann,
  dF/dc = sum v dw_ap/dc - sky dA_ap/dc - A_ap dsky/dc with
  dsky/dc = (sum m v dw_ann/dc - sky sum m dw_ann/dc) / A_ann.
  The centre derivative of an overlap area is minus the inclusion-exclusion
  of dG/dx(x, y) = sign(y) min(|y|, sqrt(r^2 - x^2)) (0 for |x| >= r), and
  the same with x and y swapped for the other axis.
"""
from __future__ import annotations

import math

import numpy as np

from .background import clip_mask
from .params import (Params, SRC_APERTURE_OFF_EDGE, SRC_ANNULUS_OFF_EDGE,
                     SRC_NO_SKY)


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------
def _P(s: float, r: float) -> float:
    return 0.5 * (s * math.sqrt(max(r * r - s * s, 0.0))
                  + r * r * math.asin(min(s / r, 1.0)))


def corner_area(x: float, y: float, r: float) -> float:
    """Signed area G(x, y) of the disk of radius r about the origin inside
    the rectangle spanned by (0, 0) and (x, y)."""
    if r <= 0.0:
        return 0.0
    sx = -1.0 if x < 0 else 1.0
    sy = -1.0 if y < 0 else 1.0
    ax, ay = min(abs(x), r), min(abs(y), r)
    if ax * ax + ay * ay <= r * r:
        a = ax * ay
    else:
        xs = math.sqrt(r * r - ay * ay)
        a = ay * xs + _P(ax, r) - _P(xs, r)
    return sx * sy * a


def touches(cx: float, cy: float, r: float, px: int, py: int) -> bool:
    """The pixel's square meets the open disk of radius r about c."""
    dx = max(abs(px - cx) - 0.5, 0.0)
    dy = max(abs(py - cy) - 0.5, 0.0)
    return dx * dx + dy * dy < r * r


def within(cx: float, cy: float, r: float, px: int, py: int) -> bool:
    """The pixel's square lies in the closed disk of radius r about c."""
    fx = abs(px - cx) + 0.5
    fy = abs(py - cy) + 0.5
    return fx * fx + fy * fy <= r * r


def overlap(cx: float, cy: float, r: float, px: int, py: int) -> float:
    """Area of disk(c, r) intersected with pixel (px, py)."""
    if not touches(cx, cy, r, px, py):
        return 0.0
    if within(cx, cy, r, px, py):
        return 1.0
    x0, x1 = px - 0.5 - cx, px + 0.5 - cx
    y0, y1 = py - 0.5 - cy, py + 0.5 - cy
    return (corner_area(x1, y1, r) - corner_area(x0, y1, r)
            - corner_area(x1, y0, r) + corner_area(x0, y0, r))


def _chord(x: float, y: float, r: float) -> float:
    """dG/dx at (x, y): signed length of [0, y] inside the circle at x."""
    if r <= 0.0 or abs(x) >= r:
        return 0.0
    h = math.sqrt(r * r - x * x)
    return math.copysign(min(abs(y), h), y)


def overlap_grad(cx: float, cy: float, r: float, px: int, py: int):
    """(d/dcx, d/dcy) of ``overlap``."""
    x0, x1 = px - 0.5 - cx, px + 0.5 - cx
    y0, y1 = py - 0.5 - cy, py + 0.5 - cy
    gx = -(_chord(x1, y1, r) - _chord(x0, y1, r) - _chord(x1, y0, r)
           + _chord(x0, y0, r))
    gy = -(_chord(y1, x1, r) - _chord(y0, x1, r) - _chord(y1, x0, r)
           + _chord(y0, x0, r))
    return gx, gy


def window(c: float, R: float):
    """Pixel indices whose extent meets [c - R, c + R]."""
    return range(math.ceil(c - R - 0.5), math.floor(c + R + 0.5) + 1)


# --------------------------------------------------------------------------
# Forward
# --------------------------------------------------------------------------
def _source_pixels(img, B, cx, cy, p: Params):
    """Weights, values and validity of every pixel of the outer window."""
    h, w = img.shape
    rows = []
    R = max(p.r_ap, p.r_out)
    for py in window(cy, R):
        for px in window(cx, R):
            in_ap = touches(cx, cy, p.r_ap, px, py)
            in_ann = (touches(cx, cy, p.r_out, px, py)
                      and not within(cx, cy, p.r_in, px, py))
            if not (in_ap or in_ann):
                continue
            wap = overlap(cx, cy, p.r_ap, px, py) if in_ap else 0.0
            wann = ((overlap(cx, cy, p.r_out, px, py)
                     - overlap(cx, cy, p.r_in, px, py)) if in_ann else 0.0)
            inside = 0 <= px < w and 0 <= py < h
            ok = inside and math.isfinite(float(img[py, px]))
            v = (float(img[py, px]) - float(B[py, px])) if ok else 0.0
            rows.append((px, py, wap, wann, ok, v, in_ap, in_ann))
    return rows


def measure(img, B, cx: float, cy: float, p: Params):
    """Photometry of one source; returns a dict with the sky mask."""
    rows = _source_pixels(img, B, cx, cy, p)
    flags = 0
    if any(r[6] and not r[4] for r in rows):
        flags |= SRC_APERTURE_OFF_EDGE
    if any(r[7] and not r[4] for r in rows):
        flags |= SRC_ANNULUS_OFF_EDGE
    ann = [r for r in rows if r[7] and r[4]]
    vals = np.array([r[5] for r in ann], dtype=np.float64)
    m = clip_mask(vals, p.sky_clip_iters, p.sky_clip_sigma)
    a_ann = math.fsum(r[3] for r, k in zip(ann, m) if k)
    if a_ann > 0:
        sky = math.fsum(r[3] * r[5] for r, k in zip(ann, m) if k) / a_ann
    else:
        sky = 0.0
        flags |= SRC_NO_SKY
    ap = [r for r in rows if r[6] and r[4]]
    a_ap = math.fsum(r[2] for r in ap)
    raw = math.fsum(r[2] * r[5] for r in ap)
    flux = raw - sky * a_ap
    return {"flux": flux, "sky": sky, "area_ap": a_ap, "area_ann": a_ann,
            "flags": flags,
            "sky_pixels": [(r[0], r[1]) for r, k in zip(ann, m) if k]}


def photometry(frame, B32, xs, ys, p: Params):
    """Aperture photometry of every (x, y); dict of arrays."""
    img = np.asarray(frame, dtype=np.float32)
    B = np.asarray(B32, dtype=np.float32)
    out = {k: [] for k in ("flux", "sky", "area_ap", "area_ann", "flags",
                           "sky_pixels")}
    for cx, cy in zip(np.asarray(xs, dtype=np.float64).tolist(),
                      np.asarray(ys, dtype=np.float64).tolist()):
        r = measure(img, B, cx, cy, p)
        for k in out:
            out[k].append(r[k])
    res = {k: np.asarray(out[k], dtype=np.float64)
           for k in ("flux", "sky", "area_ap", "area_ann")}
    res["flags"] = np.asarray(out["flags"], dtype=np.int64)
    res["sky_pixels"] = out["sky_pixels"]
    return res


# --------------------------------------------------------------------------
# Adjoint (sky clip mask held fixed)
# --------------------------------------------------------------------------
def measure_adjoint(img, B, cx: float, cy: float, p: Params, sky_pixels,
                    dLdF: float = 1.0):
    """Gradient of dLdF * flux w.r.t. the pixel values (dict (px,py)->g)
    and the centre (gx, gy), with the annulus survivors ``sky_pixels``."""
    h, w = img.shape
    keep = set(sky_pixels)
    rows = _source_pixels(img, B, cx, cy, p)
    a_ap = math.fsum(r[2] for r in rows if r[6] and r[4])
    a_ann = math.fsum(r[3] for r in rows if r[4] and (r[0], r[1]) in keep)
    sky = (math.fsum(r[3] * r[5] for r in rows
                     if r[4] and (r[0], r[1]) in keep) / a_ann
           if a_ann > 0 else 0.0)
    gv = {}
    for px, py, wap, wann, ok, v, _, _ in rows:
        if not ok:
            continue
        g = wap
        if a_ann > 0 and (px, py) in keep:
            g -= a_ap * wann / a_ann
        if g != 0.0:
            gv[(px, py)] = dLdF * g
    # centre derivative
    t_vx, t_vy, t_ax, t_ay = [], [], [], []      # aperture terms
    s_vx, s_vy, s_x, s_y = [], [], [], []        # sky terms
    for px, py, wap, wann, ok, v, _, _ in rows:
        if not ok:
            continue
        ax, ay = overlap_grad(cx, cy, p.r_ap, px, py)
        t_vx.append(v * ax)
        t_vy.append(v * ay)
        t_ax.append(ax)
        t_ay.append(ay)
        if a_ann > 0 and (px, py) in keep:
            ox, oy = overlap_grad(cx, cy, p.r_out, px, py)
            ix, iy = overlap_grad(cx, cy, p.r_in, px, py)
            bx, by = ox - ix, oy - iy
            s_vx.append(v * bx)
            s_vy.append(v * by)
            s_x.append(bx)
            s_y.append(by)
    if a_ann > 0:
        dsx = (math.fsum(s_vx) - sky * math.fsum(s_x)) / a_ann
        dsy = (math.fsum(s_vy) - sky * math.fsum(s_y)) / a_ann
    else:
        dsx = dsy = 0.0
    gx = math.fsum(t_vx) - sky * math.fsum(t_ax) - a_ap * dsx
    gy = math.fsum(t_vy) - sky * math.fsum(t_ay) - a_ap * dsy
    return gv, dLdF * gx, dLdF * gy


def photometry_adjoint(frame, B32, xs, ys, p: Params, sky_pixels, dLdF):
    """Dense dL/dv (h, w) and per-source dL/dx, dL/dy."""
    img = np.asarray(frame, dtype=np.float32)
    B = np.asarray(B32, dtype=np.float32)
    gpix = np.zeros(img.shape, dtype=np.float64)
    gx = np.zeros(len(xs))
    gy = np.zeros(len(xs))
    for k, (cx, cy) in enumerate(zip(np.asarray(xs, np.float64).tolist(),
                                     np.asarray(ys, np.float64).tolist())):
        gv, gx[k], gy[k] = measure_adjoint(img, B, cx, cy, p, sky_pixels[k],
                                           float(dLdF[k]))
        for (px, py), g in gv.items():
            gpix[py, px] += g
    return gpix, gx, gy
