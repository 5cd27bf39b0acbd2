"""Gray-scale transformations (Sec. 2.2.6) in FP64: the zscale display
range, point maps (linear, logarithmic, exponential, power law) and
histogram equalization.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names these methods and, for histogram equalization, its steps
(count the pixels of each gray level, form the cumulative distribution, and
map every pixel onto it by interpolation); it fixes no parameters.  The
readings taken, binding for the HIP kernels too:

zscale (the display-range estimate of SAOimage DS9 and IRAF):
  1. sample: the finite pixels at rows 0, s, 2s, ... and columns 0, s, 2s,
     ..., with s the smallest positive integer for which
     ceil(H/s) * ceil(W/s) <= nsamples (1000): at most nsamples values;
  2. sort the sample: v_0 <= ... <= v_{n-1}; its median per Eq. 1;
  3. fit the line v_i ~ a + b i by least squares over the samples not
     rejected (all at first); residuals r_i = v_i - (a + b i) for every
     sample; scale = ddof-0 standard deviation of the residuals of the kept
     samples; every sample with |r_i| > krej * scale is rejected, and each
     rejection spreads to the samples within ngrow // 2 indices of it
     (ngrow = max(1, floor(n / 100))); rejections are never undone.  The
     fit is repeated (at most max_iter = 5 fits) while the kept count
     falls and stays >= minpix = max(5, floor(n / 2));
  4. if the kept count is >= minpix, the line through the median at the
     central index c = floor((n - 1) / 2) with slope b' = b / contrast
     (contrast 0.25) bounds the range: z1 = max(v_0, med - c b'),
     z2 = min(v_{n-1}, med + (n - 1 - c) b'); otherwise z1 = v_0 and
     z2 = v_{n-1}.  An empty sample gives z1 = z2 = 0.

Point maps: x = (v - lo) / (hi - lo) clipped to [0, 1] (for hi <= lo,
x = 0 where v <= lo and 1 elsewhere); then linear y = x, logarithmic
y = ln(1 + a x) / ln(1 + a), exponential y = (a^x - 1) / (a - 1) and power
law y = x^a, each mapping [0, 1] onto [0, 1].  Non-finite v gives NaN.

Histogram equalization over nbins (4096) equal bins spanning the finite
pixel values [lo, hi]: the bin of v is floor(((v - lo) / (hi - lo)) nbins),
the top value going to the last bin; cdf_k = (pixels in bins 0..k) / N;
bin centres c_k = lo + (k + 1/2) (hi - lo) / nbins; y = the piecewise
linear interpolation of (c_k, cdf_k) at v, held at cdf_0 below c_0 and at
1 above the last centre.  A constant frame maps to 1; non-finite pixels
to NaN.
"""
from __future__ import annotations

import math

import numpy as np

LINEAR, LOG, EXP, POWER = 0, 1, 2, 3


# ------------------------------------------------------------------ zscale
def sample_stride(h: int, w: int, nsamples: int = 1000) -> int:
    """Smallest s >= 1 with ceil(h/s) * ceil(w/s) <= nsamples."""
    s = 1
    while -(-h // s) * -(-w // s) > nsamples:
        s += 1
    return s


def zscale_sample(frame: np.ndarray, nsamples: int = 1000) -> np.ndarray:
    """The grid sample of step 1, sorted (FP32 values as FP64)."""
    h, w = frame.shape
    s = sample_stride(h, w, nsamples)
    v = np.asarray(frame, dtype=np.float32)[::s, ::s].ravel()
    v = v[np.isfinite(v)].astype(np.float64)
    return np.sort(v)


def _median_sorted(v: np.ndarray) -> float:
    n = v.size
    if n % 2:
        return float(v[(n - 1) // 2])
    return (float(v[n // 2 - 1]) + float(v[n // 2])) / 2.0


def _line_fit(v: np.ndarray, keep: np.ndarray):
    """Least-squares line through (i, v_i) over the kept i: normal
    equations with exactly rounded sums."""
    i = np.nonzero(keep)[0]
    n = float(i.size)
    sx = math.fsum(i.astype(np.float64).tolist())
    sxx = math.fsum((i.astype(np.float64) ** 2).tolist())
    sy = math.fsum(v[i].tolist())
    sxy = math.fsum((i.astype(np.float64) * v[i]).tolist())
    den = n * sxx - sx * sx
    b = (n * sxy - sx * sy) / den if den != 0.0 else 0.0
    a = (sy - b * sx) / n
    return a, b


def zscale(frame: np.ndarray, nsamples: int = 1000, contrast: float = 0.25,
           krej: float = 2.5, max_iter: int = 5):
    """(z1, z2, info) of the frame."""
    v = zscale_sample(frame, nsamples)
    n = v.size
    if n == 0:
        return 0.0, 0.0, {"n": 0, "kept": 0, "fits": 0, "slope": 0.0}
    med = _median_sorted(v)
    minpix = max(5, n // 2)
    ngrow = max(1, n // 100)
    half = ngrow // 2
    bad = np.zeros(n, dtype=bool)
    kept, last = n, n + 1
    b = 0.0
    fits = 0
    idx = np.arange(n, dtype=np.float64)
    while fits < max_iter and kept < last and kept >= minpix:
        a, b = _line_fit(v, ~bad)
        fits += 1
        r = v - (a + b * idx)
        rk = r[~bad]
        mu = math.fsum(rk.tolist()) / rk.size
        scale = math.sqrt(math.fsum(((rk - mu) ** 2).tolist()) / rk.size)
        new = np.abs(r) > krej * scale
        grown = new.copy()
        for j in np.nonzero(new)[0]:
            grown[max(0, j - half):min(n, j + half + 1)] = True
        bad |= grown
        last, kept = kept, int(np.count_nonzero(~bad))
    z1, z2 = float(v[0]), float(v[-1])
    if kept >= minpix:
        slope = b / contrast if contrast > 0 else b
        c = (n - 1) // 2
        z1 = max(z1, med - c * slope)
        z2 = min(z2, med + (n - 1 - c) * slope)
    return z1, z2, {"n": n, "kept": kept, "fits": fits, "slope": b,
                    "median": med}


# -------------------------------------------------------------- point maps
def point_map(v, kind: int, lo: float, hi: float, a: float = 1000.0):
    v = np.asarray(v, dtype=np.float64)
    if hi > lo:
        x = np.clip((v - lo) / (hi - lo), 0.0, 1.0)
    else:
        x = np.where(v <= lo, 0.0, 1.0)
    if kind == LINEAR:
        y = x
    elif kind == LOG:
        y = np.log1p(a * x) / math.log1p(a)
    elif kind == EXP:
        y = np.expm1(x * math.log(a)) / (a - 1.0)
    elif kind == POWER:
        y = x ** a
    else:
        raise ValueError("unknown map")
    return np.where(np.isfinite(v), y, np.nan)


# -------------------------------------------------- histogram equalization
def equalize_hist(frame: np.ndarray, nbins: int = 4096):
    """(y, counts, lo, hi): y per the reading above (FP64)."""
    v = np.asarray(frame, dtype=np.float32).astype(np.float64)
    fin = np.isfinite(v)
    f = v[fin]
    counts = np.zeros(nbins, dtype=np.int64)
    y = np.full(v.shape, np.nan)
    if f.size == 0:
        return y, counts, 0.0, 0.0
    lo, hi = float(f.min()), float(f.max())
    if hi == lo:
        counts[0] = f.size
        y[fin] = 1.0
        return y, counts, lo, hi
    k = np.floor(((f - lo) / (hi - lo)) * nbins).astype(np.int64)
    k = np.minimum(k, nbins - 1)
    counts = np.bincount(k, minlength=nbins).astype(np.int64)
    cdf = np.cumsum(counts) / float(f.size)
    centres = lo + (np.arange(nbins) + 0.5) * ((hi - lo) / nbins)
    y[fin] = np.interp(f, centres, cdf)
    return y, counts, lo, hi
