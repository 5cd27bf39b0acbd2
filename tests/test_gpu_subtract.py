"""GPU parity of the stamp convolution and subtraction (Sec. 2.2.4, Eq.
8-10) against the oracle: every pixel of small frames and sampled pixels of
a 4096 x 4096 frame, within 1e-5 of the convolution's condition scale
(sum |K| |R| + |I| + |B|); spatially varying kernels, ragged stamps, frame
edges, several parameter sets and a two-frame batch."""
import math

import numpy as np
import pytest
import torch

from oracle import subtract as osb
from synth import make_frame

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _coef(rng, sp):
    """Coefficients of moderate size: each basis term scaled by
    1 / sigma^(i+j) so the kernel stays O(1) over its support."""
    terms = osb.basis_terms(sp.sigmas, sp.orders)
    ns = osb.n_poly(sp.spatial_order)
    a = []
    for s, i, j in terms:
        c = rng.normal(0, 1, ns) / (s ** (i + j) * math.factorial(i + j))
        a.append(c.tolist())
    b = rng.normal(0, 5, osb.n_poly(sp.bkg_order)).tolist()
    return a, b


def _flat(a, b):
    return np.concatenate([np.ravel(a), b]).astype(np.float64)


def _check(I, R, sp, a, b, D, pixels=None):
    Dw = osb.subtract(I, R, sp.sigmas, sp.orders, sp.half_width, a,
                      sp.spatial_order, b, sp.bkg_order, stamp=sp.stamp,
                      pixels=pixels)
    Kb = osb.basis(sp.sigmas, sp.orders, sp.half_width)
    h, w = I.shape
    pts = pixels if pixels is not None else \
        [(x, y) for y in range(h) for x in range(w)]
    worst = 0.0
    for x, y in pts:
        xs = [s for s in osb.stamps(w, sp.stamp) if s[0] <= x < s[1]][0]
        ys = [s for s in osb.stamps(h, sp.stamp) if s[0] <= y < s[1]][0]
        K = osb.stamp_kernel(Kb, a, sp.spatial_order, w, h, xs[2], ys[2])
        B = osb.poly(b, sp.bkg_order, osb.norm_coord(xs[2], w),
                     osb.norm_coord(ys[2], h))
        scale = osb.condition_scale(R, K, x, y, sp.half_width) + \
            abs(float(I[y, x])) + abs(B)
        worst = max(worst, abs(float(D[y, x]) - Dw[y, x]) / scale)
    return worst


@pytest.mark.parametrize("kw,shape", [
    (dict(), (47, 66)),
    (dict(half_width=4, stamp=8, sigmas=(1.0, 2.0), orders=(2, 1),
          spatial_order=3, bkg_order=2), (30, 41)),
    (dict(half_width=15, stamp=32, sigmas=(0.9,), orders=(7,),
          spatial_order=0, bkg_order=0), (40, 40)),
    (dict(half_width=1, stamp=1, sigmas=(0.5, 1.0, 1.5, 2.0),
          orders=(0, 1, 0, 2), spatial_order=4, bkg_order=4), (9, 7)),
    (dict(half_width=3, stamp=5), (1, 13)),
], ids=["default", "small-basis", "wide-kernel", "per-pixel", "one-row"])
def test_every_pixel_matches_the_oracle(ctx, kw, shape):
    rng = np.random.default_rng(sum(shape))
    sp = ipp.SubtractParams(**kw)
    h, w = shape
    R = rng.normal(500, 50, shape).astype(np.float32)
    I = rng.normal(480, 50, shape).astype(np.float32)
    a, b = _coef(rng, sp)
    D = ctx.subtract([torch.from_numpy(I).to(DEV)],
                     [torch.from_numpy(R).to(DEV)], sp,
                     torch.from_numpy(_flat(a, b)).to(DEV))[0]
    torch.cuda.synchronize()
    worst = _check(I, R, sp, a, b, D.cpu().numpy())
    print(f"{kw or 'default'} {shape}: worst error {worst:.2e} of scale",
          flush=True)
    assert worst <= 1e-5


def test_batch_of_two_and_a_large_frame_sampled(ctx):
    rng = np.random.default_rng(9)
    sp = ipp.SubtractParams()
    R0, _, _ = make_frame("stack16", 2)                 # 4096 x 4096 stars
    I0 = (R0.numpy() * np.float32(1.02) + np.float32(3.0)).astype(
        np.float32)
    R1 = rng.normal(300, 20, (70, 95)).astype(np.float32)
    I1 = rng.normal(310, 20, (70, 95)).astype(np.float32)
    a0, b0 = _coef(rng, sp)
    a1, b1 = _coef(rng, sp)
    coef = np.stack([_flat(a0, b0), _flat(a1, b1)])
    D = ctx.subtract([torch.from_numpy(I0).to(DEV),
                      torch.from_numpy(I1).to(DEV)],
                     [R0.to(DEV), torch.from_numpy(R1).to(DEV)], sp,
                     torch.from_numpy(coef).to(DEV))
    torch.cuda.synchronize()
    pix = [(int(x), int(y)) for x, y in
           rng.integers(0, 4096, (150, 2))] + \
        [(0, 0), (4095, 4095), (4095, 0), (20, 4084), (2047, 2048)]
    w0 = _check(I0, R0.numpy(), sp, a0, b0, D[0].cpu().numpy(), pix)
    w1 = _check(I1, R1, sp, a1, b1, D[1].cpu().numpy())
    print(f"4096^2 sampled {w0:.2e}, 70x95 every pixel {w1:.2e}", flush=True)
    assert w0 <= 1e-5 and w1 <= 1e-5


def test_argument_checks(ctx):
    sp = ipp.SubtractParams()
    f = torch.zeros((10, 10), device=DEV)
    g = torch.zeros((10, 11), device=DEV)
    n = ctx.lib.ipp_subtract_coef_count(sp.to_c())
    assert n == 49 * 6 + 3
    c = torch.zeros(n, dtype=torch.float64, device=DEV)
    with pytest.raises(ipp.IppError):
        ctx.subtract([f], [g], sp, c)
    with pytest.raises(ipp.IppError):
        ctx.subtract([f], [f], ipp.SubtractParams(half_width=16),
                     torch.zeros(1, dtype=torch.float64, device=DEV))
