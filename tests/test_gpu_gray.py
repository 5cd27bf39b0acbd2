"""GPU parity of the gray-scale transformations (Sec. 2.2.6) through the C
ABI against the oracle.

Bars: zscale sample counts, kept counts and fit counts exact, (z1, z2) to
1e-12 relative (binary64 sums in another order); point maps within 2e-6 of
the binary64 map (outputs in [0, 1], evaluated in binary32); histogram
counts exact; equalized values within 1e-6 (binary32 output of a binary64
interpolation); NaN exactly where the input is not finite.
"""
import numpy as np
import pytest
import torch

from oracle import gray as og
from synth import make_frame

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _ramp(n, extra=()):
    vals = [7 + 3 * i for i in range(n)] + list(extra)
    rng = np.random.default_rng(4)
    return rng.permutation(np.array(vals, dtype=np.float32))[None, :]


def _frames():
    """Seeded frames of the workloads at reduced size, with edge cases."""
    out = []
    a, _, _ = make_frame("single", 0, scale=0.5)              # 512 x 512
    out.append(("single-512", a.numpy()))
    b, _, _ = make_frame("stack16", 2, scale=0.1)             # 409 x 409
    b = b.numpy().copy()
    b[5:9, :] = np.nan                                        # dead rows
    b[:, 100] = np.inf
    out.append(("stack16-nan", b[:, :397].copy()))            # ragged width
    rng = np.random.default_rng(21)
    out.append(("noise", rng.normal(800.0, 25.0, (300, 333))
                .astype(np.float32)))
    out.append(("ramp", _ramp(500).reshape(20, 25).copy()))
    out.append(("ramp-outliers", _ramp(500, (1e6, 2e6, 3e6)).copy()))
    out.append(("tiny", np.array([[5.0, -2.0], [9.0, 4.0]], np.float32)))
    out.append(("const", np.full((40, 37), 12.5, np.float32)))
    out.append(("allnan", np.full((9, 13), np.nan, np.float32)))
    q = np.round(rng.normal(1000.0, 8.0, (257, 255))).astype(np.float32)
    out.append(("quantised", q))
    return out


FRAMES = _frames()


def _to_dev(frames):
    return [torch.from_numpy(np.ascontiguousarray(f)).to(DEV)
            for _, f in frames]


@pytest.mark.parametrize("contrast", [0.25, 1.0])
def test_zscale_batch(ctx, contrast):
    dev = _to_dev(FRAMES)
    z, info = ctx.zscale(dev, contrast=contrast, info=True)
    torch.cuda.synchronize()
    z, info = z.cpu().numpy(), info.cpu().numpy()
    for i, (name, f) in enumerate(FRAMES):
        z1, z2, ref = og.zscale(f, contrast=contrast)
        assert info[i, 0] == ref["n"], name
        assert info[i, 1] == ref["kept"], name
        assert info[i, 2] == ref["fits"], name
        for got, want in ((z[i, 0], z1), (z[i, 1], z2)):
            assert abs(got - want) <= 1e-12 * abs(want) + 1e-12, (name, got,
                                                                  want)


def test_zscale_exact_cases(ctx):
    """Integer ramps: every sum is exact, so the ranges are exact too."""
    f = [torch.from_numpy(FRAMES[3][1]).to(DEV),
         torch.from_numpy(FRAMES[4][1]).to(DEV)]
    z, info = ctx.zscale(f, contrast=1.0, info=True)
    torch.cuda.synchronize()
    z, info = z.cpu().numpy(), info.cpu().numpy()
    assert z[0].tolist() == [8.5, 1504.0] and info[0, 3] == 3.0
    assert z[1].tolist() == [7.0, 1513.0] and info[1, 1] == 498


@pytest.mark.parametrize("kind,a", [(ipp.IPP_MAP_LINEAR, 0.0),
                                    (ipp.IPP_MAP_LOG, 1000.0),
                                    (ipp.IPP_MAP_LOG, 0.01),
                                    (ipp.IPP_MAP_EXP, 1000.0),
                                    (ipp.IPP_MAP_EXP, 1.5),
                                    (ipp.IPP_MAP_POWER, 0.5),
                                    (ipp.IPP_MAP_POWER, 3.0)])
def test_point_maps(ctx, kind, a):
    sel = [FRAMES[i] for i in (0, 1, 2, 6, 7, 8)]
    lohi = []
    for name, f in sel:
        z1, z2, _ = og.zscale(f)
        lohi.append((z1, z2))
    lohi[3] = (12.5, 12.5)                       # degenerate: a step
    lt = torch.tensor(lohi, dtype=torch.float64, device=DEV)
    out = ctx.gray_map(_to_dev(sel), kind, lt, a)
    torch.cuda.synchronize()
    for (name, f), y, (lo, hi) in zip(sel, out, lohi):
        ref = og.point_map(f, kind, lo, hi, a)
        y = y.cpu().numpy()
        assert np.array_equal(np.isnan(y), np.isnan(ref)), name
        ok = ~np.isnan(ref)
        err = np.max(np.abs(y[ok] - ref[ok])) if ok.any() else 0.0
        assert err <= 2e-6, (name, err)


@pytest.mark.parametrize("nbins", [4096, 1000, 2])
def test_equalize_batch(ctx, nbins):
    out, cnt = ctx.equalize(_to_dev(FRAMES), nbins=nbins, counts=True)
    torch.cuda.synchronize()
    cnt = cnt.cpu().numpy().view(np.uint32)
    for i, (name, f) in enumerate(FRAMES):
        y_ref, c_ref, _, _ = og.equalize_hist(f, nbins)
        assert np.array_equal(cnt[i].astype(np.int64), c_ref), name
        y = out[i].cpu().numpy()
        assert np.array_equal(np.isnan(y), np.isnan(y_ref)), name
        ok = ~np.isnan(y_ref)
        if ok.any():
            assert np.max(np.abs(y[ok] - y_ref[ok])) <= 1e-6, name


def test_pitched_views(ctx):
    """Frames that are row-pitched views of a wider array."""
    base = np.random.default_rng(2).normal(500.0, 20.0, (130, 203)).astype(
        np.float32)
    t = torch.from_numpy(base).to(DEV)
    views = [t[:, 3:190], t[10:, :101]]
    hosts = [base[:, 3:190], base[10:, :101]]
    z = ctx.zscale(views)
    eq = ctx.equalize(views, nbins=512)
    mp = ctx.gray_map(views, ipp.IPP_MAP_LOG, z, 100.0)
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    for i, h in enumerate(hosts):
        z1, z2, _ = og.zscale(h)
        assert abs(z[i, 0] - z1) <= 1e-12 * abs(z1)
        assert abs(z[i, 1] - z2) <= 1e-12 * abs(z2)
        y_ref, _, _, _ = og.equalize_hist(h, 512)
        assert np.max(np.abs(eq[i].cpu().numpy() - y_ref)) <= 1e-6
        m_ref = og.point_map(h, og.LOG, z1, z2, 100.0)
        assert np.max(np.abs(mp[i].cpu().numpy() - m_ref)) <= 2e-6


def test_stack16_full_size(ctx):
    """The 16 x 4096^2 workload: zscale of every frame against the oracle
    (exact sample, kept and fit counts); histograms of two frames exact;
    equalized and mapped values on sampled pixels."""
    from synth import spec_for, render
    frames = [render(spec_for("stack16", i), "stack16", i,
                     torch.device(DEV))[0] for i in range(16)]
    z, info = ctx.zscale(frames, info=True)
    out, cnt = ctx.equalize(frames, counts=True)
    mp = ctx.gray_map(frames, ipp.IPP_MAP_LOG, z, 1000.0)
    torch.cuda.synchronize()
    z, info = z.cpu().numpy(), info.cpu().numpy()
    cnt = cnt.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(0)
    for i in range(16):
        f = frames[i].cpu().numpy()
        z1, z2, ref = og.zscale(f)
        assert (info[i, 0], info[i, 1], info[i, 2]) == (ref["n"], ref["kept"],
                                                        ref["fits"])
        assert abs(z[i, 0] - z1) <= 1e-12 * abs(z1)
        assert abs(z[i, 1] - z2) <= 1e-12 * abs(z2)
        if i in (0, 9):
            y_ref, c_ref, _, _ = og.equalize_hist(f)
            assert np.array_equal(cnt[i].astype(np.int64), c_ref)
            idx = rng.integers(0, f.size, 20000)
            y = out[i].cpu().numpy().ravel()[idx]
            assert np.max(np.abs(y - y_ref.ravel()[idx])) <= 1e-6
            m = mp[i].cpu().numpy().ravel()[idx]
            m_ref = og.point_map(f.ravel()[idx], og.LOG, z1, z2, 1000.0)
            assert np.max(np.abs(m - m_ref)) <= 2e-6
    del frames, out, mp
    torch.cuda.empty_cache()


def test_invalid_arguments_rejected(ctx):
    """Host-side validation of the gray-scale calls (nothing is launched)."""
    f = [torch.zeros((8, 8), dtype=torch.float32, device=DEV)]
    lohi = torch.tensor([[0.0, 1.0]], dtype=torch.float64, device=DEV)
    bad = [
        lambda: ctx.zscale(f, nsamples=0),
        lambda: ctx.zscale(f, nsamples=1001),
        lambda: ctx.zscale(f, contrast=-1.0),
        lambda: ctx.gray_map(f, 7, lohi),
        lambda: ctx.gray_map(f, ipp.IPP_MAP_LOG, lohi, a=-1.0),
        lambda: ctx.gray_map(f, ipp.IPP_MAP_EXP, lohi, a=1.0),
        lambda: ctx.gray_map(f, ipp.IPP_MAP_POWER, lohi, a=float("nan")),
        lambda: ctx.equalize(f, nbins=1),
        lambda: ctx.equalize(f, nbins=4097),
    ]
    for call in bad:
        with pytest.raises((ipp.IppError, ValueError)):
            call()
    # a valid call still works afterwards
    y = ctx.gray_map(f, ipp.IPP_MAP_LINEAR, lohi)
    torch.cuda.synchronize()
    assert float(y[0].abs().max()) == 0.0
