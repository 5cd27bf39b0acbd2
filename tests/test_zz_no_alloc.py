"""The allocation-free asinh backward (ipp_asinh_backward_noalloc, whose
block partials live in the library's static device scratch) against the
workspace-backed ipp_asinh_backward, through the C ABI: two calls in a row,
the second on a smaller input, so a stale partial left in the shared
scratch by the first call would show in the second."""
import pytest
import torch

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(n, seed):
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    v = (torch.randn(n, generator=g, dtype=torch.float64) * 300.0
         + 20.0).to(torch.float32)
    dy = torch.randn(n, generator=g, dtype=torch.float64).to(torch.float32)
    return v.to(DEV), dy.to(DEV)


def test_noalloc_equals_workspace_backward():
    ctx = ipp.Context(0)
    a, b = 30.0, 1.7
    try:
        # large enough for every one of the 2048 partial slots, then a
        # ragged small input that uses a handful of them
        for n, seed in ((4 * 256 * 2048 * 3 + 5, 1), (70001, 2)):
            v, dy = _inputs(n, seed)
            dv_ref, dab_ref = ctx.asinh_backward(v, dy, a, b)
            dv = torch.full_like(v, float("nan"))
            dab = torch.full((2,), float("nan"), dtype=torch.float64,
                             device=DEV)
            ctx.asinh_backward_noalloc(v, dy, a, b, dv=dv, dab=dab)
            torch.cuda.synchronize()
            # same kernels, same grid, fixed reduction order: identical
            assert torch.equal(dv, dv_ref), n
            assert torch.equal(dab, dab_ref), (n, dab, dab_ref)
            # and the gradient bar against a binary64 sum on the host
            vd = v.double().cpu()
            gd = dy.double().cpu()
            r = torch.sqrt(a * a + vd * vd)
            want = torch.stack([(gd * (-b) * vd / (a * r)).sum(),
                                (gd * torch.asinh(vd / a)).sum()])
            rel = (dab.cpu() - want).abs() / want.abs()
            assert float(rel.max()) <= 1e-4, rel
        # parameter gradients only (dv not written)
        v, dy = _inputs(1000, 3)
        _, dab_ref = ctx.asinh_backward(v, dy, a, b, want_dv=False)
        dab = torch.zeros(2, dtype=torch.float64, device=DEV)
        ctx.asinh_backward_noalloc(v, dy, a, b, dab=dab)
        torch.cuda.synchronize()
        assert torch.equal(dab, dab_ref)
    finally:
        ctx.close()


def test_noalloc_rejects_bad_arguments():
    ctx = ipp.Context(0)
    try:
        v, dy = _inputs(10, 4)
        with pytest.raises(ipp.IppError):
            ctx.asinh_backward_noalloc(v, dy, 0.0, 1.0)
        with pytest.raises(ipp.IppError):
            ctx.asinh_backward_noalloc(v, dy, float("inf"), 1.0)
    finally:
        ctx.close()
