"""torch.autograd.Function wrappers of the photometry and the asinh
stretch, and gradient-based centroid refinement.

Forward and backward both run in libipp's HIP kernels; these classes only
connect them to torch's autograd graph.
"""
from __future__ import annotations

import torch

from .api import Context, Params, SourceTable


def _table(x, y, frame_idx, n_frames):
    s = x.numel()
    t = SourceTable(s, n_frames, x.device)
    t.cols["frame"][:s] = frame_idx.to(torch.int32)
    t.cols["x"][:s] = x.detach().to(torch.float64)
    t.cols["y"][:s] = y.detach().to(torch.float64)
    return t


class ApertureFlux(torch.autograd.Function):
    """Sky-subtracted aperture flux (Sec. 2.2.5 photometry) of sources on a
    stack of frames.

    Inputs: frames and bkg float32 (N, H, W) on the GPU, x and y (S,)
    centroids, frame_idx (S,) the frame of each source, a Context and
    Params.  Output: flux (S,) float64.  Gradients flow to frames (dL/dI),
    bkg (-dL/dI), x and y, with the sky clip mask of the forward held fixed.
    """

    @staticmethod
    def forward(ctx, frames, bkg, x, y, frame_idx, ipp: Context,
                params: Params):
        fl = list(frames.unbind(0))
        bl = list(bkg.unbind(0))
        table = _table(x, y, frame_idx, len(fl))
        lohi = ipp.photometry(fl, bl, table, params, keep_sky=True,
                              use_count=False)
        ctx.save_for_backward(frames, bkg)
        ctx.table, ctx.lohi, ctx.ipp, ctx.params = table, lohi, ipp, params
        return table.cols["flux_ap"][:x.numel()].clone()

    @staticmethod
    def backward(ctx, g):
        frames, bkg = ctx.saved_tensors
        need_pix = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        dfr = torch.zeros_like(frames) if need_pix else None
        fl = list(frames.unbind(0))
        bl = list(bkg.unbind(0))
        dxy = ctx.ipp.photometry_backward(
            fl, bl, ctx.table, ctx.params, ctx.lohi, g.detach(),
            dpix=list(dfr.unbind(0)) if need_pix else None)
        s = g.numel()
        gx = dxy[:s, 0] if ctx.needs_input_grad[2] else None
        gy = dxy[:s, 1] if ctx.needs_input_grad[3] else None
        return (dfr if ctx.needs_input_grad[0] else None,
                -dfr if ctx.needs_input_grad[1] else None,
                gx, gy, None, None, None)


class AsinhStretch(torch.autograd.Function):
    """y = b * asinh(v / a) (Sec. 2.2.6 gray-scale map), float32 v.  a and b
    are 0-d tensors: on the GPU they are handed to the library as a device
    pair (no host round trip); Python numbers or CPU tensors are passed by
    value."""

    @staticmethod
    def forward(ctx, v, a, b, ipp: Context):
        ctx.ipp = ipp
        ctx.save_for_backward(v)
        on_dev = (isinstance(a, torch.Tensor) and a.is_cuda
                  and isinstance(b, torch.Tensor) and b.is_cuda)
        if on_dev:
            ab = torch.stack([a.detach().reshape(()),
                              b.detach().reshape(())]).to(torch.float64)
            ctx.ab = ab.contiguous()
            ctx.dtypes = (a.dtype, b.dtype)
            return ipp.asinh_dev(v, ctx.ab)
        ctx.ab = (float(a), float(b))
        ctx.dtypes = (a.dtype if isinstance(a, torch.Tensor) else None,
                      b.dtype if isinstance(b, torch.Tensor) else None)
        return ipp.asinh(v, *ctx.ab)

    @staticmethod
    def backward(ctx, g):
        (v,) = ctx.saved_tensors
        need_ab = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        if isinstance(ctx.ab, torch.Tensor):
            dv, dab = ctx.ipp.asinh_backward_dev(
                v, g.contiguous(), ctx.ab, want_dv=ctx.needs_input_grad[0],
                want_dab=need_ab)
        else:
            dv, dab = ctx.ipp.asinh_backward(
                v, g.contiguous(), *ctx.ab, want_dv=ctx.needs_input_grad[0],
                want_dab=need_ab)
        da_t, db_t = ctx.dtypes
        ga = gb = None
        if ctx.needs_input_grad[1]:
            ga = dab[0].to(da_t or torch.float32)
        if ctx.needs_input_grad[2]:
            gb = dab[1].to(db_t or torch.float32)
        return dv, ga, gb, None


def refine_centroids(ipp: Context, frames, bkg, x0, y0, frame_idx,
                     params: Params, steps: int = 10, eta: float = 3.0,
                     r_c: float = 2.0):
    """Gradient-ascent centroid refinement (ipp_refine_centroids): maximise
    F_rc(c) / F_ap(c0), the sky-subtracted flux in an aperture of radius r_c
    normalised by the flux in the default aperture at the starting point;
    c <- c + eta * grad, `steps` times.  Sources whose normaliser is <= 0
    are left in place.  Returns the refined (x, y)."""
    fl = list(frames.unbind(0))
    bl = list(bkg.unbind(0))
    s = x0.numel()
    t = _table(x0, y0, frame_idx, len(fl))
    ipp.refine_centroids(fl, bl, t, params, steps=steps, eta=eta, r_c=r_c,
                         x_out=t.cols["x"], y_out=t.cols["y"])
    return t.cols["x"][:s].clone(), t.cols["y"][:s].clone()
