"""GPU parity of deblending and cleaning (Sec. 2.2.5) against the oracle:
object maps and every column of the object table bit-exact, given the
oracle's background maps and detection.  Random blends with several
parameter sets, crowded-recipe frames, a two-frame batch, and the
capacity and scratch edges."""
import numpy as np
import pytest
import torch

import oracle
from oracle import background as obg, deblend as odb, detect as odt
from synth import make_frame

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
COLS = ("label", "npix", "xmin", "xmax", "ymin", "ymax", "peak_x", "peak_y",
        "peak", "flux_iso", "x", "y", "flags")


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _params(**kw):
    dkw = {k: kw.pop(k) for k in ("nthresh", "mincont", "clean",
                                  "clean_param") if k in kw}
    op = oracle.Params(**kw)
    for k, v in dkw.items():
        setattr(op, {"nthresh": "deblend_nthresh",
                     "mincont": "deblend_mincont",
                     "clean": "deblend_clean"}.get(k, k), v)
    return ipp.Params(**kw), ipp.DeblendParams(**dkw), op


def _run(ctx, imgs, Bs, Rs, p, dp, op):
    frames = [torch.from_numpy(i).to(DEV) for i in imgs]
    B = [torch.from_numpy(b).to(DEV) for b in Bs]
    R = [torch.from_numpy(r).to(DEV) for r in Rs]
    det = ctx.detect(frames, B, R, p,
                     capacity=sum(i.size for i in imgs) // 16 + 64)
    out = ctx.deblend(frames, B, R, det["labels"], det["table"], p, dp)
    torch.cuda.synchronize()
    return det, out


def _check(ctx, imgs, Bs, Rs, p, dp, op):
    det, out = _run(ctx, imgs, Bs, Rs, p, dp, op)
    d = out["diag"].cpu().tolist()
    assert d[2] == 0, d
    tab = out["table"].rows()
    par = out["parent"][:tab["label"].size].cpu().numpy()
    offs = out["table"].frame_offsets.cpu().numpy()
    nsplit = 0
    for i, (I, B, R) in enumerate(zip(imgs, Bs, Rs)):
        dref = odt.detect(I, B, R, op)
        ref = odb.deblend(I, B, R, dref["labels"], dref["table"], op)
        assert np.array_equal(out["objects"][i].cpu().numpy(),
                              ref["objects"]), i
        sl = slice(int(offs[i]), int(offs[i + 1]))
        assert offs[i + 1] - offs[i] == ref["n"]
        for k in COLS:
            got = tab[k][sl]
            want = ref["table"][k]
            if k != "flags":
                got = got.astype(np.float64)
            assert np.array_equal(got, want.astype(got.dtype)), (i, k)
        assert np.array_equal(par[sl], ref["table"]["parent"])
        assert np.all(tab["frame"][sl] == i)
        nsplit += int(np.count_nonzero(ref["counts"] > 1))
    assert d[3] == tab["label"].size
    return nsplit


def _blends(seed, h=96, w=128, nstar=24):
    rng = np.random.default_rng(500 + seed)
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    img = 50.0 + rng.normal(0, 1.0, (h, w))
    for _ in range(nstar):
        xc, yc = rng.uniform(3, w - 3), rng.uniform(3, h - 3)
        f = rng.uniform(30, 8000)
        s2 = rng.uniform(1.0, 3.0)
        img += f / (2 * np.pi * s2) * np.exp(-((x - xc) ** 2 +
                                                (y - yc) ** 2) / (2 * s2))
    img = img.astype(np.float32)
    return img, np.full_like(img, 50.0), np.full_like(img, 1.0)


@pytest.mark.parametrize("kw", [
    dict(det_nsigma=2.5),
    dict(det_nsigma=2.5, connectivity=4, nthresh=16, clean=0),
    dict(det_nsigma=3.0, nthresh=64, mincont=0.0005, clean_param=2.0),
    dict(det_nsigma=2.0, nthresh=2),
], ids=["default", "conn4-16-noclean", "64-lowcont", "2-levels"])
def test_random_blends(ctx, kw):
    p, dp, op = _params(min_area=3, **kw)
    nsplit = 0
    for seed in range(3):
        img, B, R = _blends(seed)
        nsplit += _check(ctx, [img], [B], [R], p, dp, op)
    assert nsplit > 0


def test_two_frame_batch_numbering(ctx):
    p, dp, op = _params(min_area=3, det_nsigma=2.5)
    a = _blends(7)
    b = _blends(8, h=70, w=61, nstar=12)
    _check(ctx, [a[0], b[0]], [a[1], b[1]], [a[2], b[2]], p, dp, op)


@pytest.mark.parametrize("frame", [2])
def test_crowded_recipe_shrunk(ctx, frame):
    img, _, _ = make_frame("crowded", frame, scale=0.15)     # 1584 x 1584
    I = img.numpy()
    p, dp, op = _params()
    ref = obg.background(I, op)
    nsplit = _check(ctx, [I], [ref["B32"]], [ref["R32"]], p, dp, op)
    print(f"crowded frame {frame} x0.15: {nsplit} split candidates",
          flush=True)
    assert nsplit > 100


def test_small_object_capacity_and_scratch_growth(ctx):
    p, dp, op = _params(min_area=3, det_nsigma=2.5)
    img, B, R = _blends(3)
    frames = [torch.from_numpy(img).to(DEV)]
    Bt = [torch.from_numpy(B).to(DEV)]
    Rt = [torch.from_numpy(R).to(DEV)]
    det = ctx.detect(frames, Bt, Rt, p, capacity=4096)
    full = ctx.deblend(frames, Bt, Rt, det["labels"], det["table"], p, dp)
    # a scratch pool far too small at first: the binding grows it
    grown = ctx.deblend(frames, Bt, Rt, det["labels"], det["table"], p, dp,
                        scratch_bytes=512)
    torch.cuda.synchronize()
    assert torch.equal(full["objects"][0], grown["objects"][0])
    n = full["table"].count()
    assert n >= 3
    # an object table smaller than the objects: the maps stay complete, the
    # count reports the need, and the rows written are the first ones
    small = ctx.deblend(frames, Bt, Rt, det["labels"], det["table"], p, dp,
                        capacity=2)
    torch.cuda.synchronize()
    assert small["table"].count() == n
    assert torch.equal(small["objects"][0], full["objects"][0])
    a = small["table"].cols["x"][:2].cpu().numpy()
    b = full["table"].cols["x"][:2].cpu().numpy()
    assert np.array_equal(a, b)
    with pytest.raises(ipp.IppError):
        ctx.deblend(frames, Bt, Rt, det["labels"], det["table"], p,
                    ipp.DeblendParams(nthresh=24))


def _plateau_spikes(h, w, boxes, seed):
    """Flat plateaus (20 sigma) carrying single-pixel spikes on a grid of
    pitch `step` ((y0, x0, size, step) per plateau; step 0: three Gaussian
    stars instead): components with many roots per level and bounding
    boxes on both sides of the wavefront / workgroup and LDS limits."""
    rng = np.random.default_rng(900 + seed)
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    img = 50.0 + rng.normal(0, 1.0, (h, w))
    for (y0, x0, n, step) in boxes:
        img[y0:y0 + n, x0:x0 + n] += 20.0
        if step == 0:
            for _ in range(3):
                xc = rng.uniform(x0 + 4, x0 + n - 4)
                yc = rng.uniform(y0 + 4, y0 + n - 4)
                img += rng.uniform(500, 5000) / (2 * np.pi * 2.0) * np.exp(
                    -((x - xc) ** 2 + (y - yc) ** 2) / 4.0)
            continue
        for yy in range(y0, y0 + n, step):
            for xx in range(x0 + (yy - y0) % 2 * (step == 1),
                            x0 + n, max(step, 2)):
                img[yy, xx] += rng.uniform(100, 5000)
    img = img.astype(np.float32)
    return img, np.full_like(img, 50.0), np.full_like(img, 1.0)


def test_large_boxes_and_many_roots(ctx):
    # a 90 x 90 plateau with 2025 spikes (box beyond the LDS arrays, more
    # roots per level than LDS holds, thousands of objects), a 40 x 40
    # plateau with three stars (a workgroup, LDS arrays) and a 20 x 20 one
    # (a wavefront)
    p, dp, op = _params(min_area=3, det_nsigma=2.5, mincont=1e-4)
    img, B, R = _plateau_spikes(
        160, 200, [(4, 4, 90, 2), (110, 110, 40, 0), (120, 20, 20, 0)], 0)
    assert _check(ctx, [img], [B], [R], p, dp, op) >= 2


def test_many_roots_in_a_small_box(ctx):
    # 4-connectivity, a 20 x 20 plateau whose spikes form a checkerboard:
    # 200 components at the spike levels in a box a wavefront takes
    p, dp, op = _params(min_area=3, det_nsigma=2.5, connectivity=4,
                        mincont=1e-4)
    img, B, R = _plateau_spikes(40, 40, [(8, 8, 20, 1)], 1)
    assert _check(ctx, [img], [B], [R], p, dp, op) >= 1
