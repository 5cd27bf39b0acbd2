"""Stamp convolution and image subtraction, Sec. 2.2.4 of the paper (Image
Subtraction Function; the kernel of Eq. 8 built from the basis of Eq. 9,
the convolution of Eq. 10), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's method (HOTPANTS): the template R is convolved with a kernel
K(u, v) = sum_n a_n(x, y) K_n(u, v), K_n(u, v) = exp(-(u^2 + v^2) /
(2 sigma_k^2)) u^i v^j (several Gaussians, each with a maximum order of
i + j), so that R (x) K = I + B (Eq. 10) for the science image I and a
background difference B; the convolution runs per stamp of 21 x 21 pixels,
with the stamp's kernel held in fast memory.  The fit of the coefficients
a_n and B from bright sources is not part of this path: they are inputs.
Readings taken here (binding for the GPU path too):

* Basis order: Gaussians in the order given; for each, i = 0 .. order and
  j = 0 .. order - i.  Offsets u (columns) and v (rows) run over
  [-hw, hw].
* Spatial variation: a_n(x, y) and B(x, y) are polynomials in normalised
  coordinates xn = (2x - (W-1)) / (W-1), yn likewise (0 for a
  one-pixel axis), sum_{p=0..d} sum_{q=0..d-p} c_pq xn^p yn^q with the
  coefficients in that order.  Each stamp uses the kernel and background
  at its centre, the centre of its actual pixel extent (partial stamps at
  the right and bottom edges are kept).
* Convolution: (R (x) K)(x, y) = sum_{u, v} K(u, v) R(x - u, y - v), with
  R = 0 outside the frame.
* Difference: D = (I + B) - R (x) K, zero where Eq. 10 holds.
"""
from __future__ import annotations

import math

import numpy as np


def n_poly(d: int) -> int:
    return (d + 1) * (d + 2) // 2


def basis_terms(sigmas, orders):
    """(sigma, i, j) of every basis function, in basis order."""
    out = []
    for s, o in zip(sigmas, orders):
        for i in range(o + 1):
            for j in range(o - i + 1):
                out.append((float(s), i, j))
    return out


def basis(sigmas, orders, hw):
    """The basis kernels K_n, shape (N, 2hw+1, 2hw+1), indexed [n, v, u]."""
    d = np.arange(-hw, hw + 1, dtype=np.float64)
    V, U = np.meshgrid(d, d, indexing="ij")
    ks = []
    for s, i, j in basis_terms(sigmas, orders):
        g = np.exp(-(U * U + V * V) / (2.0 * s * s))
        ks.append(g * U ** i * V ** j)
    return np.asarray(ks)


def norm_coord(x: float, n: int) -> float:
    return (2.0 * x - (n - 1)) / (n - 1) if n > 1 else 0.0


def poly(coef, d: int, xn: float, yn: float) -> float:
    """sum c_pq xn^p yn^q, p = 0..d, q = 0..d-p, in that order."""
    tot = 0.0
    k = 0
    for p in range(d + 1):
        for q in range(d - p + 1):
            tot += coef[k] * xn ** p * yn ** q
            k += 1
    return tot


def stamps(n: int, s: int):
    """(start, stop, centre) of each stamp along an axis of n pixels."""
    out = []
    for a in range(0, n, s):
        b = min(a + s, n)
        out.append((a, b, (a + b - 1) / 2.0))
    return out


def stamp_kernel(Kb, a_coef, spatial_order, W, H, xc, yc):
    xn, yn = norm_coord(xc, W), norm_coord(yc, H)
    a = np.array([poly(c, spatial_order, xn, yn) for c in a_coef])
    return np.tensordot(a, Kb, axes=1)


def convolve_at(R, K, x, y, hw):
    h, w = R.shape
    tot = 0.0
    for v in range(-hw, hw + 1):
        yy = y - v
        if not 0 <= yy < h:
            continue
        for u in range(-hw, hw + 1):
            xx = x - u
            if 0 <= xx < w:
                tot += K[v + hw, u + hw] * float(R[yy, xx])
    return tot


def subtract(I, R, sigmas, orders, hw, a_coef, spatial_order, b_coef,
             bkg_order, stamp=21, pixels=None):
    """Difference image D = (I + B) - R (x) K (float64), or only at the
    given (x, y) pixels when ``pixels`` is a list (the rest NaN)."""
    I = np.asarray(I, dtype=np.float32)
    R = np.asarray(R, dtype=np.float32)
    h, w = I.shape
    Kb = basis(sigmas, orders, hw)
    D = np.full((h, w), np.nan)
    want = None if pixels is None else set(map(tuple, pixels))
    for y0, y1, yc in stamps(h, stamp):
        for x0, x1, xc in stamps(w, stamp):
            if want is not None and not any(
                    x0 <= x < x1 and y0 <= y < y1 for x, y in want):
                continue
            K = stamp_kernel(Kb, a_coef, spatial_order, w, h, xc, yc)
            B = poly(b_coef, bkg_order, norm_coord(xc, w), norm_coord(yc, h))
            for y in range(y0, y1):
                for x in range(x0, x1):
                    if want is not None and (x, y) not in want:
                        continue
                    D[y, x] = (float(I[y, x]) + B) - convolve_at(R, K, x, y,
                                                                  hw)
    return D


def condition_scale(R, K, x, y, hw):
    """sum |K| |R| over the pixel's footprint: the scale of the rounding
    error of any summation order of the convolution."""
    h, w = R.shape
    tot = 0.0
    for v in range(-hw, hw + 1):
        for u in range(-hw, hw + 1):
            yy, xx = y - v, x - u
            if 0 <= yy < h and 0 <= xx < w:
                tot += abs(K[v + hw, u + hw] * float(R[yy, xx]))
    return tot
