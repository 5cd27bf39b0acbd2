"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded frames.

Bars: mesh survivor counts and medians exact, mean/sigma-derived values to
1e-12 relative; background maps <= 1e-6 relative to the oracle's binary64
map; labels and detection tables bit-exact given the same (B32, R32) maps;
aperture fluxes <= 1e-5 of the flux's condition scale.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import background as obg, detect as odt, photometry as oph
from synth import make_frame

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _params(**kw):
    return ipp.Params(**kw), oracle.Params(**kw)


def _frames():
    """(name, frame, mesh): the single-frame workload at full size, and a
    shrunken 16-frame-workload frame with ragged tiles."""
    a, _, _ = make_frame("single", 0)                       # 1024 x 1024
    b, _, _ = make_frame("stack16", 3, scale=0.0813)        # 333 x 333
    b = b[:, :317].contiguous()
    return [("single-1024", a, 64), ("stack16-ragged", b, 32)]


CASES = _frames()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mesh_and_background_parity(ctx, case):
    name, img, m = case
    p, op = _params(mesh_h=m, mesh_w=m)
    out = ctx.background([img.to(DEV)], p, mesh=True)
    torch.cuda.synchronize()
    ref = obg.background(img.numpy(), op)
    n = out["n_used"][0].cpu().numpy()
    assert np.array_equal(n, ref["n_used"]), name
    braw = out["bkg_raw"][0].cpu().numpy()
    rraw = out["rms_raw"][0].cpu().numpy()
    np.testing.assert_allclose(braw, ref["bkg_raw"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(rraw, ref["rms_raw"], rtol=1e-11, atol=0)
    np.testing.assert_allclose(out["bkg_mesh"][0].cpu().numpy(),
                               ref["bkg_mesh"], rtol=1e-12, atol=0)
    B = out["bkg"][0].cpu().numpy()
    R = out["rms"][0].cpu().numpy()
    relB = np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"]))
    relR = np.max(np.abs(R - ref["R64"]) / np.abs(ref["R64"]))
    assert relB <= 1e-6 and relR <= 1e-6, (relB, relR)
    assert int(out["flags"][0]) == ref["flags"]


def _cmp_table(tab, ref):
    for k in ("label", "npix", "xmin", "xmax", "ymin", "ymax", "peak_x",
              "peak_y", "peak", "flux_iso", "x", "y", "flags"):
        got = tab[k].astype(np.float64) if k != "flags" else tab[k]
        want = ref[k]
        assert np.array_equal(got, want.astype(got.dtype)), k


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("conn", [8, 4])
def test_detect_bit_exact_given_oracle_maps(ctx, case, conn):
    name, img, m = case
    p, op = _params(mesh_h=m, mesh_w=m, connectivity=conn)
    I = img.numpy()
    ref = obg.background(I, op)
    det = odt.detect(I, ref["B32"], ref["R32"], op)
    B = torch.from_numpy(ref["B32"]).to(DEV)
    R = torch.from_numpy(ref["R32"]).to(DEV)
    out = ctx.detect([img.to(DEV)], [B], [R], p, capacity=20000)
    torch.cuda.synchronize()
    assert int(out["diag"][2]) == 0
    tab = out["table"].rows()
    assert tab["label"].size == det["n"]
    assert np.array_equal(out["labels"][0].cpu().numpy(), det["labels"])
    _cmp_table(tab, det["table"])


def _flux_scale(ph):
    raw = ph["flux"] + ph["sky"] * ph["area_ap"]
    return np.abs(raw) + ph["area_ap"] * np.abs(ph["sky"]) + 1e-30


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_photometry_parity(ctx, case):
    name, img, m = case
    p, op = _params(mesh_h=m, mesh_w=m)
    I = img.numpy()
    ref = obg.background(I, op)
    det = odt.detect(I, ref["B32"], ref["R32"], op)
    t = det["table"]
    k = min(t["x"].size, 300)
    table = ipp.SourceTable(k, 1, DEV)
    table.cols["frame"][:k] = 0
    table.cols["x"][:k] = torch.from_numpy(t["x"][:k]).to(DEV)
    table.cols["y"][:k] = torch.from_numpy(t["y"][:k]).to(DEV)
    B = torch.from_numpy(ref["B32"]).to(DEV)
    ctx.photometry([img.to(DEV)], [B], table, p, use_count=False)
    torch.cuda.synchronize()
    got = {c: table.cols[c][:k].cpu().numpy()
           for c in ("flux_ap", "sky", "area_ap", "area_ann", "flags")}
    ph = oph.photometry(I, ref["B32"], t["x"][:k], t["y"][:k], op)
    err = np.abs(got["flux_ap"] - ph["flux"]) / _flux_scale(ph)
    assert err.max() <= 1e-5, err.max()
    np.testing.assert_allclose(got["sky"], ph["sky"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(got["area_ap"], ph["area_ap"], rtol=1e-12)
    np.testing.assert_allclose(got["area_ann"], ph["area_ann"], rtol=1e-9)
    assert np.array_equal(got["flags"], ph["flags"].astype(np.int32))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_batch_against_oracle(ctx, case):
    name, img, m = case
    p, op = _params(mesh_h=m, mesh_w=m)
    out = ctx.process_batch([img.to(DEV)], p, capacity=20000, write_rms=True)
    torch.cuda.synchronize()
    I = img.numpy()
    ref = obg.background(I, op)
    B = out["bkg"][0].cpu().numpy()
    R = out["rms"][0].cpu().numpy()
    assert np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"])) <= 1e-6
    # the oracle's detection on the GPU's own (B32, R32) is bit-exact
    det = odt.detect(I, B, R, op)
    tab = out["table"].rows()
    assert np.array_equal(out["labels"][0].cpu().numpy(), det["labels"])
    ph = oph.photometry(I, B, tab["x"], tab["y"], op)
    t = det["table"]
    for k in ("label", "npix", "flux_iso", "x", "y", "peak"):
        assert np.array_equal(tab[k], t[k].astype(tab[k].dtype)), k
    err = np.abs(tab["flux_ap"] - ph["flux"]) / _flux_scale(ph)
    assert err.max() <= 1e-5, err.max()
    # against the oracle's own maps: B32 may differ by one rounding step at
    # a few pixels, so labels agree except near those pixels
    diffB = np.count_nonzero(B != ref["B32"])
    assert diffB <= 1e-4 * B.size


def test_batch_equals_plain_per_frame(ctx):
    frames = [make_frame("uneven", i, scale=0.125)[0] for i in range(5)]
    frames += [make_frame("stack16", 1, scale=0.05)[0]]
    p = ipp.Params(mesh_h=32, mesh_w=32)
    dev = [f.to(DEV) for f in frames]
    bat = ctx.process_batch(dev, p, capacity=50000)
    torch.cuda.synchronize()
    tb = bat["table"].rows()
    offs = bat["table"].frame_offsets.cpu().numpy()
    for i, f in enumerate(dev):
        bg = ctx.background([f], p)
        d = ctx.detect([f], bg["bkg"], bg["rms"], p, capacity=20000)
        ctx.photometry([f], bg["bkg"], d["table"], p)
        torch.cuda.synchronize()
        assert torch.equal(bg["bkg"][0], bat["bkg"][i])
        assert torch.equal(d["labels"][0], bat["labels"][i])
        t = d["table"].rows()
        sl = slice(offs[i], offs[i + 1])
        for k in t:
            if k == "frame":
                assert np.all(tb[k][sl] == i)
                continue
            assert np.array_equal(t[k], tb[k][sl]), (i, k)


def test_deterministic(ctx):
    img = make_frame("stack16", 5, scale=0.1)[0].to(DEV)
    p = ipp.Params(mesh_h=32, mesh_w=32)
    a = ctx.process_batch([img], p, capacity=20000)
    b = ctx.process_batch([img], p, capacity=20000)
    torch.cuda.synchronize()
    assert torch.equal(a["bkg"][0], b["bkg"][0])
    assert torch.equal(a["labels"][0], b["labels"][0])
    ta, tb = a["table"].rows(), b["table"].rows()
    for k in ta:
        assert np.array_equal(ta[k], tb[k]), k


def test_edge_cases(ctx):
    p, op = _params(mesh_h=16, mesh_w=16)
    cases = {
        "nan": torch.full((40, 50), float("nan")),
        "const": torch.full((40, 50), 7.0),
        "tiny": make_frame("single", 0, scale=0.02)[0],       # 20 x 20
        "one_row": make_frame("single", 1, scale=0.25)[0][:1].contiguous(),
    }
    for name, img in cases.items():
        out = ctx.process_batch([img.to(DEV)], p, capacity=1000,
                                write_rms=True)
        torch.cuda.synchronize()
        ref = obg.background(img.numpy(), op)
        B = out["bkg"][0].cpu().numpy()
        assert np.allclose(B, ref["B64"], rtol=1e-6, atol=1e-9), name
        assert int(out["flags"][0]) == ref["flags"], name
        R = out["rms"][0].cpu().numpy()
        det = odt.detect(img.numpy(), B, R, op)
        assert np.array_equal(out["labels"][0].cpu().numpy(), det["labels"])
    # a table too small: labels stay complete, the count reports the need
    img = make_frame("single", 0, scale=0.25)[0].to(DEV)
    out = ctx.process_batch([img], ipp.Params(mesh_h=32, mesh_w=32),
                            capacity=3, write_rms=True)
    torch.cuda.synchronize()
    n = out["table"].count()
    assert n > 3
    assert int(out["labels"][0].max()) == n


def _mesh_variant_cases():
    img, _, _ = make_frame("single", 2, scale=0.5)             # 512 x 512
    rng = np.random.default_rng(7)
    mask = rng.random(img.shape) < 0.1
    mask[64:128, 0:128] = True                   # fully masked regions
    quant = torch.round(img / 4.0) * 4.0          # many equal values
    return [
        ("mask", img, mask, (32, 32)),
        ("mesh128", img, None, (128, 128)),
        ("mesh48x80", img, None, (48, 80)),
        ("mesh20x30", img, None, (20, 30)),
        ("quantised", quant, None, (64, 64)),
    ]


@pytest.mark.parametrize("case", _mesh_variant_cases(),
                         ids=lambda c: c[0])
def test_mesh_variants(ctx, case):
    """Masks, large and non-square regions, and heavily tied values, which
    take the other register layouts and the narrowing path of the region
    selection."""
    name, img, mask, (mh, mw) = case
    p, op = _params(mesh_h=mh, mesh_w=mw)
    masks = None
    if mask is not None:
        masks = [torch.from_numpy(mask.astype(np.uint8)).to(DEV)]
    out = ctx.background([img.to(DEV)], p, mesh=True, masks=masks)
    torch.cuda.synchronize()
    ref = obg.background(img.numpy(), op, mask)
    assert np.array_equal(out["n_used"][0].cpu().numpy(), ref["n_used"]), name
    np.testing.assert_allclose(out["bkg_raw"][0].cpu().numpy(),
                               ref["bkg_raw"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(out["rms_raw"][0].cpu().numpy(),
                               ref["rms_raw"], rtol=1e-11, atol=0)
    B = out["bkg"][0].cpu().numpy()
    assert np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"])) <= 1e-6, name


EST_CASES = [
    # (id, estimator, clip_iters, clip_sigma, median_factor, mean_factor)
    ("median-eq1", oracle.params.EST_MEDIAN, 3, 3.0, 3.0, 2.0),
    ("mean-eq2", oracle.params.EST_MEAN, 3, 3.0, 3.0, 2.0),
    ("mode-eq4", oracle.params.EST_MODE, 3, 3.0, 3.0, 2.0),
    ("mode-eq4-factors", oracle.params.EST_MODE, 3, 3.0, 2.5, 1.5),
    ("sextractor-1pass", oracle.params.EST_SEXTRACTOR, 1, 3.0, 3.0, 2.0),
    ("sextractor-0pass", oracle.params.EST_SEXTRACTOR, 0, 3.0, 3.0, 2.0),
    ("sextractor-5pass-2.5sigma", oracle.params.EST_SEXTRACTOR, 5, 2.5, 3.0,
     2.0),
    ("median-8pass-2sigma", oracle.params.EST_MEDIAN, 8, 2.0, 3.0, 2.0),
]


@pytest.mark.parametrize("case", EST_CASES, ids=lambda c: c[0])
def test_estimators_and_clip_settings(ctx, case):
    """Eq. 1, 2 and 4 and non-default clipping (passes, k) through the
    region kernel and the fused path, against the oracle."""
    name, est, iters, k, mf, af = case
    img, _, _ = make_frame("stack16", 6, scale=0.125)          # 512 x 512
    kw = dict(mesh_h=32, mesh_w=32, estimator=est, clip_iters=iters,
              clip_sigma=k, median_factor=mf, mean_factor=af)
    p, op = _params(**kw)
    out = ctx.background([img.to(DEV)], p, mesh=True)
    torch.cuda.synchronize()
    ref = obg.background(img.numpy(), op)
    assert np.array_equal(out["n_used"][0].cpu().numpy(), ref["n_used"])
    braw = out["bkg_raw"][0].cpu().numpy()
    rraw = out["rms_raw"][0].cpu().numpy()
    eb = np.max(np.abs(braw - ref["bkg_raw"]) / np.abs(ref["bkg_raw"]))
    er = np.max(np.abs(rraw - ref["rms_raw"]) / np.abs(ref["rms_raw"]))
    print(f"{name}: mesh bkg rel {eb:.2e}, rms rel {er:.2e}", flush=True)
    assert eb <= 1e-12 and er <= 1e-11, (eb, er)
    B = out["bkg"][0].cpu().numpy()
    assert np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"])) <= 1e-6
    fused = ctx.process_batch([img.to(DEV)], p, capacity=20000)
    torch.cuda.synchronize()
    assert torch.equal(fused["bkg"][0], out["bkg"][0])


def _flat_maps(h, w, b=100.0, r=10.0):
    return (np.full((h, w), np.float32(b), dtype=np.float32),
            np.full((h, w), np.float32(r), dtype=np.float32))


def _detect_vs_oracle(ctx, I, B32, R32, p, op):
    det = odt.detect(I, B32, R32, op)
    out = ctx.detect([torch.from_numpy(I).to(DEV)],
                     [torch.from_numpy(B32).to(DEV)],
                     [torch.from_numpy(R32).to(DEV)], p,
                     capacity=det["n"] + 64)
    torch.cuda.synchronize()
    tab = out["table"].rows()
    assert tab["label"].size == det["n"]
    assert np.array_equal(out["labels"][0].cpu().numpy(), det["labels"])
    _cmp_table(tab, det["table"])
    return det


def test_nonpositive_flux_branch(ctx):
    """A threshold below the sky (det_nsigma < 0) detects candidates whose
    values sum to <= 0: both sides take the unweighted centroid and flag
    the row.  A hand-built frame (sums -30 and exactly 0) and a noise frame
    with many candidates of either sign."""
    B32, R32 = _flat_maps(40, 70)
    I = B32 - 100.0
    for y, x in ((1, 1), (1, 2), (2, 1)):
        I[y, x] = 90.0
    I[5, 5], I[5, 6], I[6, 6] = 105.0, 95.0, 100.0
    p, op = _params(min_area=1, det_nsigma=-5.0)
    det = _detect_vs_oracle(ctx, I, B32, R32, p, op)
    assert det["n"] == 2
    assert all(f & oracle.params.SRC_NONPOSITIVE_FLUX
               for f in det["table"]["flags"])
    rng = np.random.default_rng(11)
    B32, R32 = _flat_maps(300, 277)
    # v ~ N(-16, 8) against t = -8: a sixth of the pixels are detected and
    # a candidate's values average about -4
    I = (B32 + rng.normal(-16.0, 8.0, B32.shape)).astype(np.float32)
    p, op = _params(det_nsigma=-0.8, min_area=3)
    det = _detect_vs_oracle(ctx, I, B32, R32, p, op)
    neg = np.count_nonzero(det["table"]["flags"]
                           & oracle.params.SRC_NONPOSITIVE_FLUX)
    print(f"noise frame: {det['n']} candidates, {neg} with sum <= 0",
          flush=True)
    assert neg > 0


def test_huge_values_are_clamped_like_the_oracle(ctx):
    """Finite values whose fixed-point weight v 2^28 reaches 2^62 are
    clamped to 2^62 - 1 on both sides (flux, centroid and moments)."""
    img, _, _ = make_frame("single", 0, scale=0.25)             # 256 x 256
    I = img.numpy().copy()
    op = oracle.Params(mesh_h=32, mesh_w=32)
    ref = obg.background(I, op)
    det0 = odt.detect(I, ref["B32"], ref["R32"], op)
    t = det0["table"]
    big = np.argsort(t["npix"])[-3:]
    for j, val in zip(big, (1e11, 2.0 ** 34, 3e38)):
        I[t["peak_y"][j], t["peak_x"][j]] = np.float32(val)
    p = ipp.Params(mesh_h=32, mesh_w=32)
    det = _detect_vs_oracle(ctx, I, ref["B32"], ref["R32"], p, op)
    flagged = det["table"]["flags"] & oracle.params.SRC_INEXACT_SUM_RANGE
    assert np.count_nonzero(flagged) >= 3
    lab = torch.from_numpy(det["labels"]).to(DEV)
    n = det["n"]
    table = ipp.SourceTable(n, 1, DEV)
    for c in ("label", "xmin", "xmax", "ymin", "ymax"):
        table.cols[c][:n] = torch.from_numpy(
            det["table"][c].astype(np.int32)).to(DEV)
    table.n_total.fill_(n)
    mom = ctx.source_moments([torch.from_numpy(I).to(DEV)],
                             [torch.from_numpy(ref["B32"]).to(DEV)], [lab],
                             table).cpu().numpy()
    want = odt.source_moments(I, ref["B32"], det["labels"], n)
    ok = ~np.isnan(want[:, 0])
    assert np.array_equal(np.isnan(mom), np.isnan(want))
    assert np.array_equal(mom[ok, :3], want[ok, :3])
