"""A batch of many tiny frames of mixed shapes (down to 1 x 1, smaller than
one mesh region and one detection tile) through the batched path: per
frame, the background against the oracle (<= 1e-6), labels and the table
against the oracle's detection on the GPU's maps (bit-exact), and the
photometry (<= 1e-5)."""
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


def _frames(n, seed=31):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = (1, 1) if i == 0 else tuple(rng.integers(1, 71, 2))
        img = rng.normal(500.0, 8.0, (h, w))
        for _ in range(int(rng.integers(0, 4))):
            cy, cx = rng.integers(0, h), rng.integers(0, w)
            img[max(0, cy - 1):cy + 2, max(0, cx - 1):cx + 2] += 400.0
        out.append(img.astype(np.float32))
    return out


def test_many_small_frames(ctx):
    imgs = _frames(300)
    kw = dict(mesh_h=16, mesh_w=16)
    p, op = ipp.Params(**kw), oracle.Params(**kw)
    dev = [torch.from_numpy(f).to(DEV) for f in imgs]
    out = ctx.process_batch(dev, p, capacity=20000, write_rms=True)
    torch.cuda.synchronize()
    assert int(out["diag"][2]) == 0
    rows = out["table"].rows()
    offs = out["table"].frame_offsets.cpu().numpy()
    for i, img in enumerate(imgs):
        ref = obg.background(img, op)
        B = out["bkg"][i].cpu().numpy()
        R = out["rms"][i].cpu().numpy()
        assert int(out["flags"][i]) == ref["flags"], i
        assert np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"])) <= 1e-6, i
        det = odt.detect(img, B, R, op)
        assert np.array_equal(out["labels"][i].cpu().numpy(), det["labels"]), i
        part = {k: v[offs[i]:offs[i + 1]] for k, v in rows.items()}
        assert part["label"].size == det["n"], i
        for k in ("npix", "xmin", "xmax", "ymin", "ymax", "flux_iso", "x",
                  "y"):
            assert np.array_equal(part[k].astype(np.float64),
                                  det["table"][k].astype(np.float64)), (i, k)
        if det["n"]:
            ph = oph.photometry(img, B, part["x"], part["y"], op)
            ok = np.isfinite(ph["flux"])
            assert np.array_equal(np.isfinite(part["flux_ap"]), ok), i
            raw = ph["flux"] + ph["sky"] * ph["area_ap"]
            scale = np.abs(raw) + ph["area_ap"] * np.abs(ph["sky"]) + 1e-30
            err = np.abs(part["flux_ap"][ok] - ph["flux"][ok]) / scale[ok]
            assert err.size == 0 or err.max() <= 1e-5, i
