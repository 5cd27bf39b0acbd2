"""Multi-threshold deblending and cleaning of detection candidates, Sec.
2.2.5 of the paper (the deblending and cleaning phases), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper describes the phases as SExtractor's: each candidate's peak value
sets a series of deblending thresholds between the detection threshold and
the peak; at each threshold the candidate's pixels above it are connected
again, which splits the candidate into sub-objects and builds a tree rooted
at the candidate; the tree is walked from the bottom up and pruned by an
intensity criterion, the branches that survive being separate objects; in
cleaning, an object that can be merged with a neighbour under a fixed
criterion is taken as a false detection and its pixels go to that
neighbour.  The paper gives no formulas; the readings taken here (binding
for the GPU path too) are:

* Levels.  t0 = nsigma * (double)R32 at the candidate's peak pixel (the
  table's peak, ties to the lowest raster index).  With N = ``nthresh`` (a
  power of two) the ratio q = (peak / t0)^(1/N) is taken by log2(N)
  successive square roots and the levels are t_i = t_{i-1} * q for
  i = 1 .. N-1: every step is one correctly rounded binary64 operation.
  Candidates with t0 <= 0 or of one pixel are not deblended.
* Tree.  At level i the candidate's pixels with v > t_i form components
  (the detection's connectivity); each lies inside one component of level
  i-1 (its parent); the candidate itself is the root at level 0.
* Intensity criterion.  A node's flux is the sum of v over its pixels, an
  exact sum of the source table's fixed-point weights D = v 2^28 rounded
  once to binary64; a node is significant iff its flux exceeds
  ``mincont`` times the candidate's flux (binary64 product).
* Pruning, from the deepest level up.  A leaf is one object.  A node with
  at least two significant children stands for the objects of those
  children; with one significant child, for that child's objects if it
  has two or more, else for itself; with none, for itself.  The candidate
  splits iff its root stands for two or more objects; the objects' seeds
  are the pixels of their nodes, numbered in raster order of each seed's
  first pixel.
* Remaining pixels.  Each candidate pixel outside every seed goes to the
  seed whose model is brightest there: a Moffat profile of index 2 with the
  seed's flux F, its flux-weighted barycentre (xc, yc) and scale
  s2 = x2 + y2 + 1/6 (its second moments x2, y2 as in the moments of the
  source table, plus the variance of a uniform unit pixel on each axis):
  score = (F s2) / ((s2 + d2) (s2 + d2)), d2 = (x - xc)^2 + (y - yc)^2;
  equal scores go to the lower seed index.  Only rational operations, so
  both sides decide identically.
* Cleaning.  For object o with final pixels P_o, the mean value
  mu_o = S_o / |P_o| (exact sum, rounded) is compared with the light that
  brighter objects m of the same candidate (larger seed flux; equal flux
  and lower index) put at o's seed barycentre, c_m = k_c F_m s2_m /
  (pi (s2_m + d2)^2) (the same profile normalised to flux F_m), summed in
  index order: if mu_o - sum c_m < t0, o is merged into the m with the
  largest c_m (ties to the lower index).  Merges follow their targets to
  an object that is not merged (targets are brighter, so chains end).
  The surviving objects keep their relative order.
* Output.  Objects of one frame are numbered candidate by candidate (in
  label order), and within a candidate in seed order: an object map of the
  frame (0 outside every candidate) and the source table of that map
  (the pre-analysis of ``detect.source_table``) with the parent candidate
  of each object and a BLENDED flag on objects of a split candidate.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage

from .detect import source_table
from .params import Params, SRC_BLENDED

_Q = 28
_DMAX = (1 << 62) - 1
_SIXTH = 1.0 / 6.0


def fixed_weight(v: float) -> int:
    """The exact-sum weight D = round(v 2^28), clamped to +-(2^62 - 1)."""
    d = int(round(v * 2.0 ** _Q))
    if d > _DMAX:
        return _DMAX
    if d < -_DMAX:
        return -_DMAX
    return d


def levels(t0: float, peak: float, nthresh: int):
    """Deblending levels t_1 .. t_{N-1} (binary64, see the module text)."""
    k = int(round(math.log2(nthresh)))
    assert 1 << k == nthresh, "nthresh must be a power of two"
    q = peak / t0
    for _ in range(k):
        q = math.sqrt(q)
    out = []
    t = t0
    for _ in range(1, nthresh):
        t = t * q
        out.append(t)
    return out


def _components(mask: np.ndarray, connectivity: int):
    st = np.ones((3, 3), dtype=bool) if connectivity == 8 else None
    lab, n = scipy.ndimage.label(mask, structure=st)
    return lab, n


class _Node:
    __slots__ = ("level", "pix", "flux", "children")

    def __init__(self, level, pix, flux):
        self.level = level
        self.pix = pix              # flat indices into the bounding box
        self.flux = flux            # intensity above the node's level (ADU)
        self.children = []


def _seed_model(pix, D, bw, x0, y0):
    """Flux (ADU), barycentre and Moffat scale of a seed from exact sums
    about the seed's bounding-box corner."""
    ys, xs = pix // bw, pix % bw
    sxm, sym = int(xs.min()), int(ys.min())
    S = Sx = Sy = Sxx = Syy = 0
    for d, x, y in zip(D[pix].tolist(), xs.tolist(), ys.tolist()):
        dx, dy = x - sxm, y - sym
        S += d
        Sx += d * dx
        Sy += d * dy
        Sxx += d * dx * dx
        Syy += d * dy * dy
    fS = float(S)
    mx = float(Sx) / fS
    my = float(Sy) / fS
    x2 = float(Sxx) / fS - mx * mx
    y2 = float(Syy) / fS - my * my
    return {"F": fS * 2.0 ** -_Q,
            "xc": float(x0 + sxm) + mx, "yc": float(y0 + sym) + my,
            "s2": (x2 + y2) + _SIXTH, "first": int(pix.min())}


def deblend_candidate(v, D, member, x0, y0, t0, peak, p: Params):
    """Split one candidate.  v, D: binary64 values and integer weights over
    its bounding box (row-major, D an object array of Python ints), member:
    its pixels, (x0, y0): the box corner.  Returns (objects, assign) with
    one dict per object (seed order) and, per box pixel, the object index
    (-1 outside the candidate)."""
    bh, bw = member.shape
    flat_m = member.ravel()
    idx_all = np.nonzero(flat_m)[0]
    assign = np.full(bh * bw, -1, dtype=np.int64)
    single = [{"first": int(idx_all.min())}]
    if not (t0 > 0.0) or idx_all.size < 2 or not (peak > t0):
        assign[idx_all] = 0
        return single, assign.reshape(bh, bw)
    Dl = D.ravel()
    vl = v.ravel()
    froot = float(sum(Dl[idx_all].tolist())) * 2.0 ** -_Q
    fmin = p.deblend_mincont * froot
    root = _Node(0, idx_all, froot)
    prev_lab = None
    prev_nodes = {}
    for i, t in enumerate(levels(t0, peak, p.deblend_nthresh), start=1):
        above = flat_m & (vl > t)
        if not above.any():
            break
        lab, n = _components(above.reshape(bh, bw), p.connectivity)
        lab = lab.ravel()
        nodes = {}
        order = np.argsort(lab, kind="stable")
        starts = np.searchsorted(lab[order], np.arange(n + 2))
        for c in range(1, n + 1):
            pix = order[starts[c]:starts[c + 1]]
            above_t = (float(sum(Dl[pix].tolist())) * 2.0 ** -_Q
                       - float(pix.size) * t)
            node = _Node(i, pix, above_t)
            parent = root if prev_lab is None else \
                prev_nodes[int(prev_lab[pix[0]])]
            parent.children.append(node)
            nodes[c] = node
        prev_lab, prev_nodes = lab, nodes

    def objs(node):
        sig = [c for c in node.children if c.flux > fmin]
        sub = [objs(c) for c in sig]
        if len(sig) >= 2:
            return [o for s in sub for o in s]
        if len(sig) == 1 and len(sub[0]) >= 2:
            return sub[0]
        return [node]

    seeds = objs(root)
    if len(seeds) < 2:
        assign[idx_all] = 0
        return single, assign.reshape(bh, bw)
    seeds.sort(key=lambda nd: int(nd.pix.min()))
    model = [_seed_model(nd.pix, Dl, bw, x0, y0) for nd in seeds]
    for k, nd in enumerate(seeds):
        assign[nd.pix] = k
    rest = idx_all[assign[idx_all] < 0]
    for q in rest.tolist():
        x = float(x0 + q % bw)
        y = float(y0 + q // bw)
        best, bk = -1.0, -1
        for k, m in enumerate(model):
            dx = x - m["xc"]
            dy = y - m["yc"]
            d2 = dx * dx + dy * dy
            den = m["s2"] + d2
            sc = (m["F"] * m["s2"]) / (den * den)
            if sc > best:
                best, bk = sc, k
        assign[q] = bk
    if p.deblend_clean:
        assign = _clean(model, assign, idx_all, Dl, t0, p.clean_param)
    kept = sorted(set(assign[idx_all].tolist()))
    remap = {k: j for j, k in enumerate(kept)}
    assign[idx_all] = [remap[k] for k in assign[idx_all].tolist()]
    return [model[k] for k in kept], assign.reshape(bh, bw)


def _clean(model, assign, idx_all, Dl, t0, k_c):
    """Cleaning pass over the objects of one split candidate."""
    n = len(model)
    target = list(range(n))
    for o in range(n):
        pix = idx_all[assign[idx_all] == o]
        mu = float(sum(Dl[pix].tolist())) * 2.0 ** -_Q / float(pix.size)
        xo, yo = model[o]["xc"], model[o]["yc"]
        tot, best, bm = 0.0, -1.0, -1
        for m in range(n):
            if m == o:
                continue
            brighter = (model[m]["F"] > model[o]["F"]
                        or (model[m]["F"] == model[o]["F"] and m < o))
            if not brighter:
                continue
            dx = xo - model[m]["xc"]
            dy = yo - model[m]["yc"]
            d2 = dx * dx + dy * dy
            den = model[m]["s2"] + d2
            den = den * den
            den = math.pi * den
            c = k_c * ((model[m]["F"] * model[m]["s2"]) / den)
            tot += c
            if c > best:
                best, bm = c, m
        if bm >= 0 and mu - tot < t0:
            target[o] = bm
    final = []
    for o in range(n):
        k = o
        while target[k] != k:
            k = target[k]
        final.append(k)
    out = assign.copy()
    out[idx_all] = [final[k] for k in assign[idx_all].tolist()]
    return out


def deblend(frame, B32, R32, labels, table, p: Params):
    """Deblend and clean every candidate of one frame.  labels and table are
    the detection's (``detect.detect``).  Returns the object map (int32,
    objects numbered 1..K candidate by candidate), the object count, the
    source table of the object map with ``parent`` (the candidate label of
    each object) and BLENDED flags, and the per-candidate object counts."""
    I = np.asarray(frame, dtype=np.float32)
    B = np.asarray(B32, dtype=np.float32)
    R = np.asarray(R32, dtype=np.float32)
    h, w = labels.shape
    objmap = np.zeros((h, w), dtype=np.int32)
    counts = []
    nobj = 0
    for k in range(table["label"].size):
        lab = int(table["label"][k])
        x0, x1 = int(table["xmin"][k]), int(table["xmax"][k])
        y0, y1 = int(table["ymin"][k]), int(table["ymax"][k])
        member = labels[y0:y1 + 1, x0:x1 + 1] == lab
        v = (I[y0:y1 + 1, x0:x1 + 1].astype(np.float64)
             - B[y0:y1 + 1, x0:x1 + 1].astype(np.float64))
        D = np.empty(v.shape, dtype=object)
        D[...] = 0
        D[member] = [fixed_weight(a) for a in v[member].tolist()]
        px, py = int(table["peak_x"][k]), int(table["peak_y"][k])
        t0 = p.det_nsigma * float(R[py, px])
        objs, assign = deblend_candidate(v, D, member, x0, y0, t0,
                                         float(table["peak"][k]), p)
        sub = objmap[y0:y1 + 1, x0:x1 + 1]
        sub[member] = (nobj + 1 + assign[member]).astype(np.int32)
        counts.append(len(objs))
        nobj += len(objs)
    t = source_table(I, B, objmap, nobj)
    parent = np.repeat(table["label"], counts) if nobj else \
        np.zeros(0, dtype=np.int64)
    split = np.repeat(np.asarray(counts) > 1, counts) if nobj else \
        np.zeros(0, dtype=bool)
    t["parent"] = parent.astype(np.int64)
    t["flags"] = t["flags"] | np.where(split, SRC_BLENDED, 0)
    return {"objects": objmap, "n": nobj, "table": t,
            "counts": np.asarray(counts, dtype=np.int64)}
