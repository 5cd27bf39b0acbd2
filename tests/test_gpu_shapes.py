"""GPU parity on frames at the size limits of the ABI: rows and columns of
the largest accepted length (32767) and frames one pixel thin, through the
background (<= 1e-6 of the oracle's binary64 map), detection given the
oracle's maps (labels and table bit-exact) and photometry (<= 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import background as obg, detect as odt, photometry as oph

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _frame(h, w, seed):
    """Noise on a sloped sky with a few bright blobs (seeded)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w]
    sky = 1000.0 + 0.01 * xx + 0.02 * yy
    img = rng.normal(sky, 10.0)
    for _ in range(40):
        cy, cx = rng.integers(0, h), rng.integers(0, w)
        img[max(0, cy - 1):cy + 2, max(0, cx - 1):cx + 2] += rng.uniform(
            200.0, 2000.0)
    return img.astype(np.float32)


SHAPES = [(3, 32767), (32767, 3), (1, 5000), (5000, 1), (67, 32767)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_extreme_shapes(ctx, shape):
    h, w = shape
    img = _frame(h, w, h * 7 + w)
    kw = dict(mesh_h=32, mesh_w=32)
    p, op = ipp.Params(**kw), oracle.Params(**kw)
    fr = torch.from_numpy(img).to(DEV)
    bg = ctx.background([fr], p)
    torch.cuda.synchronize()
    ref = obg.background(img, op)
    B = bg["bkg"][0].cpu().numpy()
    assert int(bg["flags"][0]) == ref["flags"]
    assert np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"])) <= 1e-6
    det = odt.detect(img, ref["B32"], ref["R32"], op)
    Bt = torch.from_numpy(ref["B32"]).to(DEV)
    Rt = torch.from_numpy(ref["R32"]).to(DEV)
    out = ctx.detect([fr], [Bt], [Rt], p, capacity=20000)
    torch.cuda.synchronize()
    assert int(out["diag"][2]) == 0
    assert np.array_equal(out["labels"][0].cpu().numpy(), det["labels"])
    tab = out["table"].rows()
    assert tab["label"].size == det["n"]
    for k in ("npix", "xmin", "xmax", "ymin", "ymax", "flux_iso", "x", "y"):
        assert np.array_equal(tab[k].astype(np.float64),
                              det["table"][k].astype(np.float64)), k
    if det["n"]:
        ctx.photometry([fr], [Bt], out["table"], p)
        torch.cuda.synchronize()
        rows = out["table"].rows()
        ph = oph.photometry(img, ref["B32"], rows["x"], rows["y"], op)
        assert np.array_equal(rows["flags"] & 3, ph["flags"] & 3)
        ok = np.isfinite(ph["flux"])
        raw = ph["flux"] + ph["sky"] * ph["area_ap"]
        scale = np.abs(raw) + ph["area_ap"] * np.abs(ph["sky"]) + 1e-30
        err = np.abs(rows["flux_ap"][ok] - ph["flux"][ok]) / scale[ok]
        assert err.size == 0 or err.max() <= 1e-5
