"""The photometry written by the centroid refinement's first evaluation
(IPP_F_REFINE_PHOTOMETRY: the normaliser's aperture at the starting centre,
over that evaluation's sky, Sec. 2.2.5 per-object photometry) against the
photometry call on the same table: fluxes, sky, areas to rounding, flags
exactly; the refined centres are unchanged by the flag; and a batch with
IPP_F_NO_PHOTOMETRY leaves the photometry columns alone and everything else
as the full batch writes it."""
import numpy as np
import pytest
import torch

from synth import make_frame

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PHOT = ("flux_ap", "sky", "area_ap", "area_ann")


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch(ctx):
    frames = [make_frame("crowded", i, scale=0.1)[0].to(DEV)
              for i in range(2)]                          # 1056 x 1056
    p = ipp.Params()
    npx = sum(f.numel() for f in frames)
    table = ipp.SourceTable(npx // 64 + 1024, len(frames), DEV)
    out = {"bkg": [torch.empty_like(f) for f in frames],
           "labels": [torch.empty(f.shape, dtype=torch.int32, device=DEV)
                      for f in frames], "rms": None}
    ctx.process_batch(frames, p, table=table, outputs=out)
    torch.cuda.synchronize()
    n = table.count()
    assert 500 < n <= table.capacity
    return frames, out, p, table, n


def _copy(table, n, frames):
    t = ipp.SourceTable(table.capacity, len(frames), DEV)
    for k, v in table.cols.items():
        t.cols[k].copy_(v)
    t.n_total.copy_(table.n_total)
    t.frame_offsets.copy_(table.frame_offsets)
    return t


@pytest.mark.parametrize("steps", [0, 3])
def test_refinement_photometry_matches_photometry(ctx, batch, steps):
    frames, out, p, table, n = batch
    ref = _copy(table, n, frames)
    ctx.photometry(frames, out["bkg"], ref, p)
    got = _copy(table, n, frames)
    for k in PHOT:
        got.cols[k].fill_(-12345.0)
    got.cols["flags"].copy_(table.cols["flags"])
    xw, yw = ctx.refine_centroids(frames, out["bkg"], got, p, steps=steps,
                                  use_count=True, write_photometry=True)
    plain = _copy(table, n, frames)
    xp, yp = ctx.refine_centroids(frames, out["bkg"], plain, p, steps=steps,
                                  use_count=True)
    torch.cuda.synchronize()
    # the flag adds writes only: the trajectories are the same bits
    assert torch.equal(xw[:n], xp[:n]) and torch.equal(yw[:n], yp[:n])
    if steps == 0:
        assert torch.equal(xw[:n], table.cols["x"][:n])
    r = {k: ref.cols[k][:n].cpu().numpy() for k in PHOT + ("flags",)}
    g = {k: got.cols[k][:n].cpu().numpy() for k in PHOT + ("flags",)}
    assert np.array_equal(g["flags"], r["flags"])
    ok = np.isfinite(r["flux_ap"])
    assert np.array_equal(ok, np.isfinite(g["flux_ap"]))
    vmax = float(max(f.abs().max().item() for f in frames))
    for k in ("area_ap", "area_ann"):
        np.testing.assert_allclose(g[k], r[k], rtol=1e-12, atol=1e-12)
    scale = np.abs(r["flux_ap"][ok]) + r["area_ap"][ok] * vmax
    err = np.abs(g["flux_ap"][ok] - r["flux_ap"][ok]) / scale
    assert err.max() <= 1e-12
    sk = np.abs(g["sky"][ok] - r["sky"][ok]) / (np.abs(r["sky"][ok]) + vmax)
    assert sk.max() <= 1e-12


def test_batch_without_photometry(ctx, batch):
    frames, out, p, table, n = batch
    t = ipp.SourceTable(table.capacity, len(frames), DEV)
    for k in PHOT:
        t.cols[k].fill_(-12345.0)
    o2 = {"bkg": [torch.empty_like(f) for f in frames],
          "labels": [torch.empty(f.shape, dtype=torch.int32, device=DEV)
                     for f in frames], "rms": None}
    ctx.process_batch(frames, p, table=t, outputs=o2, photometry=False)
    torch.cuda.synchronize()
    assert t.count() == n
    for k in PHOT:
        assert torch.all(t.cols[k] == -12345.0), k
    for k, v in table.cols.items():
        if k in PHOT or k == "flags":
            continue
        assert torch.equal(t.cols[k][:n], v[:n]), k
    for a, b in zip(o2["labels"], out["labels"]):
        assert torch.equal(a, b)
