"""GPU tests of the pipeline-mode machinery: captured-graph replay, uneven
batches, the autotuner and its cache."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import background as obg, detect as odt
from synth import make_frame

import paper_2502_10783_amd as ipp

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = ipp.Context(0)
    yield c
    c.close()


def _uneven(n, scale, start=0):
    return [make_frame("uneven", i, scale=scale)[0] for i in
            range(start, start + n)]


def _plain(ctx, f, p):
    bg = ctx.background([f], p)
    d = ctx.detect([f], bg["bkg"], bg["rms"], p, capacity=200000)
    ctx.photometry([f], bg["bkg"], d["table"], p)
    torch.cuda.synchronize()
    return bg["bkg"][0], d["labels"][0], d["table"].rows()


def _check_against_plain(ctx, frames, out, p):
    tb = out["table"].rows()
    offs = out["table"].frame_offsets.cpu().numpy()
    for i, f in enumerate(frames):
        b, lab, t = _plain(ctx, f, p)
        assert torch.equal(b, out["bkg"][i]), i
        assert torch.equal(lab, out["labels"][i]), i
        sl = slice(offs[i], offs[i + 1])
        for k in t:
            if k != "frame":
                assert np.array_equal(t[k], tb[k][sl]), (i, k)


def test_graph_replay_with_new_data(ctx):
    p = ipp.Params(mesh_h=32, mesh_w=32)
    a = [f.to(DEV) for f in _uneven(4, 0.125)]
    b = [f.to(DEV) for f in _uneven(4, 0.125, start=40)]
    shapes = [tuple(f.shape) for f in a]
    b = [make_frame("uneven", 40 + i, scale=0.125, h=s[0], w=s[1])[0]
         .to(DEV) for i, s in enumerate(shapes)]
    table = ipp.SourceTable(100000, 4, DEV)
    outs = {"bkg": [torch.empty_like(f) for f in a],
            "labels": [torch.empty(f.shape, dtype=torch.int32, device=DEV)
                       for f in a], "rms": None}
    ctx.process_batch(a, p, table=table, outputs=outs)      # capture
    ctx.process_batch(a, p, table=table, outputs=outs)      # replay
    torch.cuda.synchronize()
    _check_against_plain(ctx, a, outs, p)
    out_b = ctx.process_batch(b, p, table=table, outputs=outs)  # new data
    torch.cuda.synchronize()
    _check_against_plain(ctx, b, out_b, p)


def test_uneven_batch_against_plain_and_oracle(ctx):
    frames = [f.to(DEV) for f in _uneven(12, 0.25)]
    p = ipp.Params()
    out = ctx.process_batch(frames, p, capacity=400000, write_rms=True)
    torch.cuda.synchronize()
    assert int(out["diag"][2]) == 0
    _check_against_plain(ctx, frames, out, p)
    # the smallest frame end to end against the oracle
    i = int(np.argmin([f.numel() for f in frames]))
    I = frames[i].cpu().numpy()
    ref = obg.background(I, oracle.Params())
    B = out["bkg"][i].cpu().numpy()
    R = out["rms"][i].cpu().numpy()
    assert np.max(np.abs(B - ref["B64"]) / np.abs(ref["B64"])) <= 1e-6
    det = odt.detect(I, B, R, oracle.Params())
    assert np.array_equal(out["labels"][i].cpu().numpy(), det["labels"])


def test_profiled_eager_equals_graph(ctx):
    frames = [f.to(DEV) for f in _uneven(3, 0.125, start=7)]
    p = ipp.Params(mesh_h=32, mesh_w=32)
    g = ctx.process_batch(frames, p, capacity=50000)
    ctx.profile(True)
    e = ctx.process_batch(frames, p, capacity=50000)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    assert "k_tile_ccl_fused" in prof and "k_mesh_stats" in prof
    for i in range(3):
        assert torch.equal(g["bkg"][i], e["bkg"][i])
        assert torch.equal(g["labels"][i], e["labels"][i])
    tg, te = g["table"].rows(), e["table"].rows()
    for k in tg:
        assert np.array_equal(tg[k], te[k]), k


def test_autotune_and_cache(ctx, tmp_path):
    frames = [f.to(DEV) for f in _uneven(6, 0.125, start=3)]
    cache = str(tmp_path / "tune.json")
    p, ms = ctx.autotune(frames, ipp.Params(), cache_path=cache)
    assert p.mesh_h in (32, 64, 128) and p.mesh_w == p.mesh_h
    assert (p.tile_h, p.tile_w) in ((64, 64), (32, 128), (128, 32))
    assert ms > 0
    data = json.load(open(cache))
    assert len(data) == 1
    entry = list(data.values())[0]
    assert (entry["mesh_h"], entry["tile_h"]) == (p.mesh_h, p.tile_h)
    p2, ms2 = ctx.autotune(frames, ipp.Params(), cache_path=cache)
    assert (p2.mesh_h, p2.tile_h, p2.tile_w) == (p.mesh_h, p.tile_h,
                                                 p.tile_w)
    assert abs(ms2 - ms) < 1e-5
    # tile shape only: results identical across shapes
    outs = []
    for th, tw in ((64, 64), (32, 128), (128, 32)):
        q = ipp.Params(tile_h=th, tile_w=tw)
        outs.append(ctx.process_batch(frames, q, capacity=50000))
    torch.cuda.synchronize()
    for o in outs[1:]:
        for i in range(len(frames)):
            assert torch.equal(o["labels"][i], outs[0]["labels"][i])
            assert torch.equal(o["bkg"][i], outs[0]["bkg"][i])
        assert np.array_equal(o["table"].rows()["flux_ap"],
                              outs[0]["table"].rows()["flux_ap"])


def test_repeated_batches_keep_their_flag_buffers(ctx):
    """The frame flags and diagnostics are overwritten by every call, so a
    caller's output dict keeps the same buffers (and device addresses, which
    the captured graph's signature includes) from call to call."""
    img = make_frame("stack16", 2, scale=0.05)[0].to(DEV)
    p = ipp.Params(mesh_h=32, mesh_w=32)
    out = ctx.process_batch([img], p, capacity=5000)
    f0, d0 = out["flags"].data_ptr(), out["diag"].data_ptr()
    lab0 = out["labels"][0].clone()
    for _ in range(3):
        out = ctx.process_batch([img], p, table=out["table"], outputs=out)
    torch.cuda.synchronize()
    assert out["flags"].data_ptr() == f0 and out["diag"].data_ptr() == d0
    assert torch.equal(out["labels"][0], lab0)
