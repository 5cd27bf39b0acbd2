"""The library's per-candidate deblending routine (deblend_core.h, the code
the GPU kernel runs per candidate), compiled for the host, against the
deblending oracle (Sec. 2.2.5), candidate by candidate: the object count
and every member pixel's object must be identical.  Runs without a GPU:
hipcc builds the host harness in _build/."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import background as obg, deblend as db, detect as dt
from synth import make_frame

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "deblend_host.cpp")
HDR = os.path.join(ROOT, "paper_2502_10783_amd", "csrc", "deblend_core.h")
LIB = os.path.join(ROOT, "_build", "libdeblend_host.so")


@pytest.fixture(scope="module")
def lib():
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not available")
    stale = (not os.path.exists(LIB) or
             os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                         os.path.getmtime(HDR)))
    if stale:
        os.makedirs(os.path.dirname(LIB), exist_ok=True)
        subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2",
                        "-fPIC", "-shared", "-std=c++17",
                        "-ffp-contract=off", SRC, "-o", LIB], check=True,
                       capture_output=True)
    L = C.CDLL(LIB)
    L.db_candidate.restype = C.c_int
    L.db_candidate.argtypes = [C.c_void_p] + [C.c_int] * 5 + \
        [C.c_double] * 2 + [C.c_int] * 3 + [C.c_double] * 2 + [C.c_void_p]
    return L


def _compare_frame(L, I, B32, R32, p, limit=None):
    det = dt.detect(I, B32, R32, p)
    t = det["table"]
    lab = det["labels"]
    Bv = np.asarray(B32, np.float32).astype(np.float64)
    Iv = np.asarray(I, np.float32).astype(np.float64)
    nsplit = 0
    n = det["n"] if limit is None else min(limit, det["n"])
    for k in range(n):
        x0, x1 = int(t["xmin"][k]), int(t["xmax"][k])
        y0, y1 = int(t["ymin"][k]), int(t["ymax"][k])
        member = lab[y0:y1 + 1, x0:x1 + 1] == k + 1
        v = Iv[y0:y1 + 1, x0:x1 + 1] - Bv[y0:y1 + 1, x0:x1 + 1]
        val = np.where(member, v, -np.inf).astype(np.float64)
        val = np.ascontiguousarray(val)
        px, py = int(t["peak_x"][k]), int(t["peak_y"][k])
        t0 = p.det_nsigma * float(np.float32(R32[py, px]))
        peak = float(t["peak"][k])
        asg = np.empty(val.shape, dtype=np.int32)
        got = L.db_candidate(val.ctypes.data, val.shape[1], val.shape[0],
                             x0, y0, int(t["npix"][k]), t0, peak,
                             p.connectivity, p.deblend_nthresh,
                             int(p.deblend_clean), p.deblend_mincont,
                             p.clean_param, asg.ctypes.data)
        D = np.empty(v.shape, dtype=object)
        D[...] = 0
        D[member] = [db.fixed_weight(a) for a in v[member].tolist()]
        objs, want = db.deblend_candidate(v, D, member, x0, y0, t0, peak, p)
        assert got == len(objs), (k, got, len(objs))
        assert np.array_equal(np.where(member, asg, -1),
                              np.where(member, want, -1)), k
        nsplit += got > 1
    return n, nsplit


@pytest.mark.parametrize("seed", range(6))
def test_random_blends(lib, seed):
    rng = np.random.default_rng(100 + seed)
    h, w = 64, 80
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    img = 50.0 + rng.normal(0, 1.0, (h, w))
    for _ in range(12):
        xc, yc = rng.uniform(4, w - 4), rng.uniform(4, h - 4)
        f = rng.uniform(30, 5000)
        img += f / (2 * np.pi * 2.0) * np.exp(-((x - xc) ** 2 +
                                                 (y - yc) ** 2) / 4.0)
    img = img.astype(np.float32)
    B = np.full_like(img, 50.0)
    R = np.full_like(img, 1.0)
    for conn, nthresh, clean in ((8, 32, True), (4, 16, False),
                                 (8, 64, True)):
        p = oracle.Params(det_nsigma=2.5, connectivity=conn,
                          deblend_nthresh=nthresh, deblend_clean=clean)
        n, nsplit = _compare_frame(lib, img, B, R, p)
        assert n > 0


def test_crowded_frame_shrunk(lib):
    img, _, _ = make_frame("crowded", 1, scale=0.1)      # 1056 x 1056
    I = img.numpy()
    p = oracle.Params()
    ref = obg.background(I, p)
    n, nsplit = _compare_frame(lib, I, ref["B32"], ref["R32"], p)
    assert nsplit > 100


def test_mincont_and_clean_variants(lib):
    img, _, _ = make_frame("stack16", 4, scale=0.08)     # 328 x 328
    I = img.numpy()
    for mc, kc in ((0.0005, 1.0), (0.05, 3.0), (0.005, 0.2)):
        p = oracle.Params(mesh_h=32, mesh_w=32, deblend_mincont=mc,
                          clean_param=kc)
        ref = obg.background(I, p)
        _compare_frame(lib, I, ref["B32"], ref["R32"], p)
