"""GPU labelling and pre-analysis (Sec. 2.2.5) on handcrafted and dense
detection patterns, bit-exact against the oracle.

Each image is a pattern mask times small integer values (10..17 ADU) over a
zero background map and a unit rms map, so that at 1.5 sigma a pixel is
detected exactly where the mask is set.  Labels and every table column
(npix, bounding box, peak and its position, iso flux, barycentre, flags)
must equal the oracle's.

The patterns stress what natural frames rarely reach: random masks near
and above the 8-neighbour site-percolation threshold; a square spiral with
one-pixel walls that winds through every tile of the frame; checkerboards
(one component under 8-connectivity, every detected pixel its own
component under 4-connectivity, which fills a tile's component table);
diagonal chains across tile seams; rows and columns that run through whole
tile rows; a fully detected and an empty frame; 4- and 5-pixel blobs on
tile seams at minimum area 5.  Frame sizes are not multiples of the tile,
and the three tile shapes are covered.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import detect as odt

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
H, W = 200, 333


def _spiral(h, w):
    """A turtle walk that turns right whenever the cell after the next one
    is already drawn or the next one is off the frame: a single winding
    component whose parallel walls are one pixel apart."""
    m = np.zeros((h, w), dtype=bool)
    y, x, dy, dx = 0, 0, 0, 1
    m[0, 0] = True

    def can_step(y, x, dy, dx):
        ny, nx = y + dy, x + dx
        if not (0 <= ny < h and 0 <= nx < w) or m[ny, nx]:
            return False
        fy, fx = ny + dy, nx + dx
        return not (0 <= fy < h and 0 <= fx < w and m[fy, fx])

    stuck = 0
    while stuck < 2:
        if can_step(y, x, dy, dx):
            y, x = y + dy, x + dx
            m[y, x] = True
            stuck = 0
        else:
            dy, dx = dx, -dy
            stuck += 1
    return m


def _blobs(h, w):
    """2x2 squares (4 px) and plus signs (5 px) centred on tile seams."""
    m = np.zeros((h, w), dtype=bool)
    for k, (cy, cx) in enumerate([(63, 63), (64, 128), (127, 200),
                                  (128, 64), (31, 255), (160, 319),
                                  (100, 31), (191, 96)]):
        if k % 2 == 0:
            m[cy:cy + 2, cx:cx + 2] = True
        else:
            m[cy, cx - 1:cx + 2] = True
            m[cy - 1:cy + 2, cx] = True
    return m


def _patterns():
    rng = np.random.default_rng(2502)
    yy, xx = np.mgrid[0:H, 0:W]
    pats = {
        "random-0.07": rng.random((H, W)) < 0.07,
        "random-0.41": rng.random((H, W)) < 0.41,
        "random-0.60": rng.random((H, W)) < 0.60,
        "spiral": _spiral(H, W),
        "checker": (yy + xx) % 2 == 0,
        "diagonals": (xx - yy) % 7 == 0,
        "rows": yy % 3 == 0,
        "columns": xx % 2 == 0,
        "full": np.ones((H, W), dtype=bool),
        "empty": np.zeros((H, W), dtype=bool),
        "blobs": _blobs(H, W),
    }
    vals = (10 + rng.integers(0, 8, (H, W))).astype(np.float32)
    return {k: (m * vals).astype(np.float32) for k, m in pats.items()}


PATTERNS = _patterns()
# (pattern, connectivity, min_area, tile shape)
CASES = [
    ("random-0.07", 8, 1, (64, 64)),
    ("random-0.41", 8, 1, (64, 64)),
    ("random-0.41", 4, 1, (64, 64)),
    ("random-0.41", 8, 5, (32, 128)),
    ("random-0.60", 8, 5, (128, 32)),
    ("random-0.60", 4, 5, (64, 64)),
    ("spiral", 8, 5, (64, 64)),
    ("spiral", 4, 5, (32, 128)),
    ("checker", 8, 5, (64, 64)),
    ("checker", 4, 1, (64, 64)),
    ("checker", 4, 1, (128, 32)),
    ("diagonals", 8, 5, (64, 64)),
    ("diagonals", 4, 1, (32, 128)),
    ("rows", 8, 5, (128, 32)),
    ("columns", 4, 5, (32, 128)),
    ("full", 8, 5, (64, 64)),
    ("empty", 8, 5, (64, 64)),
    ("blobs", 8, 5, (64, 64)),
    ("blobs", 4, 4, (32, 128)),
]


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _params(conn, min_area, tile):
    kw = dict(connectivity=conn, min_area=min_area, det_nsigma=1.5)
    return (ipp.Params(tile_h=tile[0], tile_w=tile[1], **kw),
            oracle.Params(**kw))


def _cmp_table(tab, ref):
    for k in ("label", "npix", "xmin", "xmax", "ymin", "ymax", "peak_x",
              "peak_y", "peak", "flux_iso", "x", "y", "flags"):
        got = tab[k].astype(np.float64) if k != "flags" else tab[k]
        assert np.array_equal(got, ref[k].astype(got.dtype)), k


def _run(ctx, imgs, p):
    """Detection of the frames against zero background and unit rms, with
    room for one record and one table row per pixel."""
    frames = [torch.from_numpy(i).to(DEV) for i in imgs]
    bkg = [torch.zeros_like(f) for f in frames]
    rms = [torch.ones_like(f) for f in frames]
    npx = sum(i.size for i in imgs)
    ctx.ensure(frames, p, record_capacity=npx)
    out = ctx.detect(frames, bkg, rms, p, capacity=npx)
    torch.cuda.synchronize()
    assert int(out["diag"][2]) == 0, "record capacity overflowed"
    return out


@pytest.mark.parametrize("case", CASES,
                         ids=["%s-c%d-a%d-%dx%d" % (c[0], c[1], c[2], *c[3])
                              for c in CASES])
def test_patterns_bit_exact(ctx, case):
    name, conn, amin, tile = case
    img = PATTERNS[name]
    p, op = _params(conn, amin, tile)
    out = _run(ctx, [img], p)
    z = np.zeros_like(img)
    ref = odt.detect(img, z, np.ones_like(img), op)
    tab = out["table"].rows()
    assert tab["label"].size == ref["n"]
    assert np.array_equal(out["labels"][0].cpu().numpy(), ref["labels"])
    _cmp_table(tab, ref["table"])


def test_patterns_in_one_batch(ctx):
    """All patterns as one uneven batch (cropped to different sizes):
    per-frame labels, per-frame numbering and the table's frame offsets."""
    names = sorted(PATTERNS)
    imgs = [np.ascontiguousarray(PATTERNS[k][:H - 7 * j, :W - 13 * j])
            for j, k in enumerate(names)]
    p, op = _params(8, 3, (64, 64))
    out = _run(ctx, imgs, p)
    tab = out["table"].rows()
    offs = out["table"].frame_offsets.cpu().numpy()
    for i, img in enumerate(imgs):
        ref = odt.detect(img, np.zeros_like(img), np.ones_like(img), op)
        assert np.array_equal(out["labels"][i].cpu().numpy(),
                              ref["labels"]), names[i]
        assert offs[i + 1] - offs[i] == ref["n"], names[i]
        part = {k: v[offs[i]:offs[i + 1]] for k, v in tab.items()}
        assert np.all(part["frame"] == i)
        _cmp_table(part, ref["table"])
