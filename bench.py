#!/usr/bin/env python
"""Throughput of the pre-processing hot path on one MI355X.

Default workload: the crowded large-format batch, 32 synthetic float32
frames of 10560 x 10560 (1500 ADU sky plus a 1/f^2 Gaussian random field
nebulosity of rms 100 ADU, 100k Moffat stars of beta 2.5 per frame, Poisson
and read noise, saturation at 65535), resident in HBM before the timed
region.  One step = background estimation + detection + pre-analysis +
aperture photometry of the whole batch (one fused pipeline call), then
gradient centroid refinement of every detected candidate (10 ascent steps,
each a photometry forward and backward, in one library call).

Reported on one JSON line: the batched path (value, Mpix/s; sources/s) and
the plain per-frame path (one call per step and frame, with a host sync
for the source count), their ratio, the step's algorithmic HBM bandwidth,
the roofline of the dominant kernel (HIP events recorded by the library on
the launch stream), the flux error of sampled sources against the FP64
oracle, the oracle's own throughput on a bounded sample on the host CPU
(one core and all cores), and the same batched-vs-plain figures for the
16 x 4096^2 stack and the autotuned 256-frame uneven batch.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2]
    python bench.py --workload stack16|uneven|grad64|gray16|next16
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Mpix/s and sources/s, batched+fused vs plain per-frame, at "
          "<=1e-5 flux error")
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
REFINE_STEPS = 10
REFINE_RC = 2.0
REFINE_ETA = 3.0

# Algorithmic HBM bytes of each per-pixel kernel per pixel of the batch:
# what the step must move through that kernel, not what the implementation
# moves.
ALGO_BYTES_PER_PX = {
    "k_mesh_stats": 4.0,        # read every pixel once
    "k_tile_ccl_fused": 8.0,    # read the pixel, write the background map
    "k_relabel": 4.0,           # write the label map
    "k_bkg_maps": 8.0,          # write background and rms maps
    "k_tile_ccl": 12.0,         # read pixel, background and rms maps
}
# The photometry kernels are binary64 geometry: flops per source.
ALU_KERNELS = ("k_aperture", "k_aperture_bwd", "k_refine")


def aperture_flops_per_source(r_ap, r_in, r_out):
    """Algorithmic binary64 work of one source's photometry (forward or
    backward): the pixels cut by the three circles (a circle of radius r
    crosses about 8 r unit pixels) times about 60 flops of exact-overlap
    geometry each."""
    return 60.0 * 8.0 * (r_ap + r_in + r_out)


def kron_flops(mom, kron_r):
    """Algorithmic binary64 work of AUTO photometry over its sources: the
    pixels that the Kron ellipse cuts (about 4 (A + B) for semi-axes A, B,
    as a circle of radius r cuts about 8 r) times the circle overlap's ~60
    flops plus 8 for the affine map of a pixel's corners.  A, B: the Kron
    radius times the square roots of the eigenvalues of the moments'
    covariance regularised by 1/12 on each axis."""
    import numpy as np
    X = mom[:, 0] + 1.0 / 12.0
    Y = mom[:, 1] + 1.0 / 12.0
    xy = mom[:, 2]
    tr, det = X + Y, X * Y - xy * xy
    disc = np.sqrt(np.maximum(tr * tr / 4.0 - det, 0.0))
    l1, l2 = tr / 2.0 + disc, np.maximum(tr / 2.0 - disc, 0.0)
    ab = kron_r * (np.sqrt(l1) + np.sqrt(l2))
    ok = np.isfinite(ab)
    return float(68.0 * 4.0 * ab[ok].sum())


def step_algo_bytes(npx, nsrc, refine_steps):
    """Algorithmic HBM bytes of one step: read I, write the background and
    label maps (12 B/px), one 80-byte table row per source, and per
    refinement step the positions read and written (16 B/source)."""
    return 12.0 * npx + 80.0 * nsrc + 16.0 * nsrc * refine_steps


# HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE, scaled by a copy kernel of known size), keyed by kernel with
# a hash of the sources they were measured on: reported only while the
# sources are unchanged.
def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def measured_traffic(kernel, workload):
    import hashlib
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    t = json.load(open(path)).get(kernel)
    if not t:
        return None
    h = hashlib.sha256()
    for f in t["sources"]:
        path = os.path.join(ROOT, "paper_2502_10783_amd", "csrc", f)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    if h.hexdigest()[:16] != t["source_sha256_16"]:
        return None
    return {"read_bytes": t["read_bytes"], "write_bytes": t["write_bytes"],
            "total_bytes": t["read_bytes"] + t["write_bytes"]}


def roofline(kern, dom, npx, flops_total):
    """Roofline entry of a kernel from its event-timed launches: achieved =
    algorithmic bytes (or flops) of its launches over their summed
    duration, i.e. the per-launch average over the average launch time."""
    k = kern[dom]
    ms_tot, nl = k["ms_total"], k["launches"]
    if dom in ALGO_BYTES_PER_PX:
        algo = ALGO_BYTES_PER_PX[dom] * npx
        gbs = algo * nl / (ms_tot * 1e-3) / 1e9
        return {"kernel": dom, "bound": "hbm", "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "algo_bytes_per_launch": algo,
                "ms_per_launch": round(ms_tot / nl, 4), "launches": nl}
    if dom in ALU_KERNELS and flops_total.get(dom):
        tfs = flops_total[dom] / (ms_tot * 1e-3) / 1e12
        return {"kernel": dom, "bound": "alu", "achieved": round(tfs, 4),
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfs / FP64_VECTOR_PEAK_TFLOPS, 5),
                "traffic": None,
                "algo_flops_per_launch": flops_total[dom] / nl,
                "ms_per_launch": round(ms_tot / nl, 4), "launches": nl}
    return {"kernel": dom, "bound": None, "achieved": None, "peak": None,
            "unit": None, "frac": None, "traffic": None}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_frames(workload, n, device):
    from synth import spec_for, render
    frames = []
    for i in range(n):
        img, _ = render(spec_for(workload, i), workload, i, device)
        frames.append(img)
    return frames


WORKLOADS = {
    "crowded": (32, "32 frames of 10560x10560 float32, 1/f^2 Gaussian "
                    "random field nebulosity, 100k Moffat stars each, "
                    "saturated at 65535; batched forward plus centroid "
                    "refinement (10 gradient steps) of every candidate"),
    "stack16": (16, "16 frames of 4096x4096 float32, 5000 Moffat stars each, "
                    "poly+sinusoid sky, cosmic rays, dead columns"),
    "uneven": (256, "256 float32 frames drawn from {512x512, 1024x1024, "
                    "2048x4096, 4096x4096}, star density log-uniform "
                    "1e-5..5e-3 per px, flat sky U(200, 5000); mesh and "
                    "tile shape from the autotuner"),
}
# Workloads whose step includes the centroid refinement.
REFINED = {"crowded"}


# ---------------------------------------------------------------- CPU leg
def _oracle_sample(args):
    """One bounded oracle run (worker process): background, detection and
    photometry of a shrunken frame of the workload, and the refinement of
    `k` of its sources (the rest extrapolated from their time)."""
    workload, frame, scale, k_refine = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle
    from oracle import background as obg, detect as odt, photometry as oph
    from oracle.refine import refine_centroids
    from synth import make_frame
    img, _, _ = make_frame(workload, frame, scale=scale)
    I = img.numpy()
    op = oracle.Params()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ref = obg.background(I, op)
        det = odt.detect(I, ref["B32"], ref["R32"], op)
        t = det["table"]
        oph.photometry(I, ref["B32"], t["x"], t["y"], op)
        t1 = time.perf_counter()
        k = min(k_refine, det["n"]) if k_refine else 0
        if k:
            sel = np.linspace(0, det["n"] - 1, k).astype(int)
            refine_centroids(I, ref["B32"], t["x"][sel], t["y"][sel], op,
                             steps=REFINE_STEPS, r_c=REFINE_RC)
        t2 = time.perf_counter()
    per_src_refine = (t2 - t1) / k if k else 0.0
    return {"px": I.size, "sources": det["n"], "measured_s": t2 - t0,
            "forward_s": t1 - t0,
            "total_s": (t1 - t0) + per_src_refine * det["n"]}


def cpu_baseline(workload, scale, k_refine, workers):
    """The FP64 oracle on shrunken frames of the workload (the same sky,
    noise, star density and source mix; rendered on the host): one frame on
    one core, then `workers` frames in parallel processes, one per core.
    Refinement time is measured on a sample of sources and extrapolated to
    all of them (labelled)."""
    import multiprocessing as mp
    one = _oracle_sample((workload, 0, scale, k_refine))
    desc = (f"frames of the {workload} recipe shrunk {scale}x per axis "
            f"({one['px']} px and {one['sources']} sources in frame 0): "
            f"background, detection and photometry of each")
    if k_refine:
        desc += (f", and refinement ({REFINE_STEPS} steps) of {k_refine} "
                 f"sampled sources per frame, its time per source "
                 f"extrapolated to all of the frame's sources")
    one_core = {"value": round(one["px"] / 1e6 / one["total_s"], 4),
                "unit": "Mpix/s", "cores": 1,
                "sources_per_s": round(one["sources"] / one["total_s"], 2),
                "frames": 1, "seconds_measured": round(one["measured_s"], 2)}
    res = dict(one_core, kind="oracle", sample=desc,
               host_cpu_count=os.cpu_count(), extrapolated=bool(k_refine))
    if workers > 1:
        mpc = mp.get_context("spawn")
        jobs = [(workload, i, scale, k_refine) for i in range(workers)]
        t0 = time.perf_counter()
        with mpc.Pool(workers) as pool:
            outs = pool.map(_oracle_sample, jobs)
        wall = time.perf_counter() - t0
        # each worker's extrapolated refinement added to the wall time
        span = wall + max(o["total_s"] - o["measured_s"] for o in outs)
        px = sum(o["px"] for o in outs)
        ns = sum(o["sources"] for o in outs)
        res.update({"value": round(px / 1e6 / span, 4), "cores": workers,
                    "sources_per_s": round(ns / span, 2), "frames": workers,
                    "seconds_measured": round(wall, 2),
                    "one_core": one_core})
    return res
GRAD_DESC = ("64 frames of 2048x2048 float32, 2000 Gaussian stars each, "
             "centroid guesses = truth + N(0, 0.3^2) px per axis")


def run_grad(args):
    """The differentiable part: forward + backward of the aperture flux for
    every centroid guess of the 64-frame stack (one refinement step, Sec.
    2.2.5 photometry with its adjoint), and the asinh stretch forward +
    backward over the stack (Sec. 2.2.6 gray-scale map)."""
    import torch
    import paper_2502_10783_amd as ipp
    from synth import spec_for, render

    dev = torch.device("cuda:0")
    n = args.frames or 64
    log(f"generating {n} frames of grad64 on the GPU")
    rend = [render(spec_for("grad64", i), "grad64", i, dev) for i in range(n)]
    frames = [r[0] for r in rend]
    xg = torch.cat([r[1]["x_guess"] for r in rend]).to(torch.float64)
    yg = torch.cat([r[1]["y_guess"] for r in rend]).to(torch.float64)
    fi = torch.cat([torch.full((r[1]["x_guess"].numel(),), k,
                               dtype=torch.int32, device=dev)
                    for k, r in enumerate(rend)])
    s = xg.numel()
    p = ipp.Params()
    ctx = ipp.Context(0)
    out = ctx.process_batch(frames, p)
    bkg = out["bkg"]
    t = ipp.SourceTable(s, n, dev)
    t.cols["frame"][:s] = fi
    t.cols["x"][:s] = xg
    t.cols["y"][:s] = yg
    g = torch.ones(s, dtype=torch.float64, device=dev)

    def step():
        lohi = ctx.photometry(frames, bkg, t, p, keep_sky=True,
                              use_count=False)
        return ctx.photometry_backward(frames, bkg, t, p, lohi, g)

    v = torch.stack(frames) - torch.stack(bkg)
    dy = torch.ones_like(v)
    a, b = 30.0, 1.0
    xr = torch.empty(s, dtype=torch.float64, device=dev)
    yr = torch.empty_like(xr)

    def refine():
        ctx.refine_centroids(frames, bkg, t, p, steps=REFINE_STEPS,
                             r_c=REFINE_RC, eta=REFINE_ETA, x_out=xr,
                             y_out=yr)
    if args.calib_copy:
        calibration_copy(args.calib_copy, dev)

    def timed(fn, k):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    log(f"timing {args.steps} forward+backward photometry steps")
    ms = timed(step, args.steps)
    ms_fwd = timed(lambda: ctx.asinh(v, a, b), args.steps)
    ms_bwd = timed(lambda: ctx.asinh_backward(v, dy, a, b), args.steps)
    ms_ref = timed(refine, args.steps)
    ctx.profile(True)
    for _ in range(3):
        step()
        ctx.asinh(v, a, b)
        ctx.asinh_backward(v, dy, a, b)
        refine()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    npx = v.numel()
    res = {
        "metric": "sources/s, aperture flux forward + backward (one "
                  "refinement step)",
        "value": round(s / (ms * 1e-3), 1),
        "unit": "sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": GRAD_DESC if n == 64 else
                   f"first {n} frames of: {GRAD_DESC}", "name": "grad64",
                   "frames": n, "sources": s,
                   "aperture": [p.r_ap, p.r_in, p.r_out]},
        "asinh": {
            "forward_ms": round(ms_fwd, 4),
            "forward_GBps": round(8 * npx / (ms_fwd * 1e-3) / 1e9, 1),
            "backward_ms": round(ms_bwd, 4),
            "backward_GBps": round(12 * npx / (ms_bwd * 1e-3) / 1e9, 1),
            "backward_frac_of_hbm": round(
                12 * npx / (ms_bwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_px": {"forward": 8, "backward": 12}},
        "refinement": {
            "steps": REFINE_STEPS, "r_c": REFINE_RC, "eta": REFINE_ETA,
            "ms": round(ms_ref, 4),
            "sources_per_s": round(s / (ms_ref * 1e-3), 1)},
        "kernels_ms": {k: round(v0 / v1, 4) for k, (v0, v1) in
                       sorted(prof.items(), key=lambda kv: -kv[1][0])},
    }
    print(json.dumps(res), flush=True)


SUB_DESC = ("16 pairs of 4096x4096 float32 frames (science and template of "
            "the 16-frame recipe), 21x21 kernels of 3 Gaussians (sigma 0.7, "
            "1.5, 3.0 px; orders 6, 4, 2: 49 basis terms) with degree-2 "
            "spatial coefficients and a degree-1 background, 21x21 stamps")
FP32_VECTOR_PEAK_TFLOPS = 157.3


def _sub_coef(nfr, sp, seed=7):
    """Seeded kernel and background coefficients of moderate size (each
    basis term scaled by 1 / (sigma^(i+j) (i+j)!), so that the kernel stays
    O(1) over its support); the fit that would produce them is not part of
    the path."""
    import math
    import numpy as np
    rng = np.random.default_rng(seed)
    ns = (sp.spatial_order + 1) * (sp.spatial_order + 2) // 2
    nb = (sp.bkg_order + 1) * (sp.bkg_order + 2) // 2
    rows = []
    for _ in range(nfr):
        a = []
        for s, o in zip(sp.sigmas, sp.orders):
            for i in range(o + 1):
                for j in range(o - i + 1):
                    a.append(rng.normal(0, 1, ns) /
                             (s ** (i + j) * math.factorial(i + j)))
        a.append(rng.normal(0, 5, nb))
        rows.append(np.concatenate(a))
    return np.stack(rows)


def _next_cpu_sample(args):
    """The oracle on small pieces of the 16-frame recipe (one process):
    stamp subtraction of a 24 x 24 crop, deblending and cleaning of the
    candidates of a 512 x 512 crop, AUTO photometry of 50 of them."""
    import time as _t
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle
    from oracle import background as obg, detect as odt, deblend as odb
    from oracle import kron as okr, subtract as osb
    from synth import make_frame
    from paper_2502_10783_amd.api import SubtractParams
    frame = args
    with threadpool_limits(1):
        img, _, _ = make_frame("stack16", frame, scale=0.125)   # 512 x 512
        I = img.numpy()
        op = oracle.Params()
        sp = SubtractParams()
        coef = _sub_coef(1, sp, seed=frame)[0]
        ns = (sp.spatial_order + 1) * (sp.spatial_order + 2) // 2
        nbt = len(osb.basis_terms(sp.sigmas, sp.orders))
        a = coef[:nbt * ns].reshape(nbt, ns)
        b = coef[nbt * ns:]
        crop = 96
        t0 = _t.perf_counter()
        osb.subtract(I[:crop, :crop], I[1:crop + 1, 1:crop + 1], sp.sigmas,
                     sp.orders, sp.half_width, a, sp.spatial_order, b,
                     sp.bkg_order, stamp=sp.stamp)
        t_sub = _t.perf_counter() - t0
        ref = obg.background(I, op)
        det = odt.detect(I, ref["B32"], ref["R32"], op)
        t0 = _t.perf_counter()
        odb.deblend(I, ref["B32"], ref["R32"], det["labels"], det["table"],
                    op)
        t_db = _t.perf_counter() - t0
        k = min(200, det["n"])
        t0 = _t.perf_counter()
        mom = odt.source_moments(I, ref["B32"], det["labels"], det["n"])
        okr.auto_photometry(I, ref["B32"], det["table"]["x"][:k],
                            det["table"]["y"][:k], mom[:k])
        t_auto = _t.perf_counter() - t0
    return {"sub_px": crop * crop, "sub_s": t_sub, "db_px": I.size,
            "db_s": t_db, "auto_src": k, "auto_s": t_auto}


def run_next(args):
    """The widened rows on the 16-frame stack: deblending and cleaning of
    the detection's candidates (Sec. 2.2.5), second moments and AUTO
    photometry of the candidates (Sec. 2.2.5, 3.3) and the stamp
    convolution and difference image against a template (Sec. 2.2.4)."""
    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline of the widened rows (one core)")
        t0 = time.time()
        r = _next_cpu_sample(0)
        cpu = {"kind": "oracle", "cores": 1,
               "sample": ("frame 0 of the 16-frame recipe shrunk to "
                          "512x512: stamp subtraction of a 96x96 crop, "
                          "deblending and cleaning of all its candidates, "
                          "moments and AUTO photometry of 200 of them"),
               "subtract_mpix_per_s": round(r["sub_px"] / r["sub_s"] / 1e6,
                                            6),
               "deblend_mpix_per_s": round(r["db_px"] / r["db_s"] / 1e6, 4),
               "auto_sources_per_s": round(r["auto_src"] / r["auto_s"], 2),
               "seconds_measured": round(time.time() - t0, 1)}
    import torch
    import paper_2502_10783_amd as ipp
    from paper_2502_10783_amd.api import SubtractParams
    dev = torch.device("cuda:0")
    nfr, desc = WORKLOADS["stack16"]
    if args.frames:
        nfr = min(nfr, args.frames)
    log(f"generating {nfr} frames of stack16 on the GPU")
    frames = make_frames("stack16", nfr, dev)
    templates = [torch.roll(f, shifts=(1, 1), dims=(0, 1)).contiguous()
                 for f in frames]
    if args.calib_copy:
        calibration_copy(args.calib_copy, dev)
    npx = sum(f.numel() for f in frames)
    ctx = ipp.Context(0)
    p = ipp.Params()
    table = ipp.SourceTable(npx // 64 + 4096, nfr, dev)
    outputs = {"bkg": [torch.empty_like(f) for f in frames],
               "labels": [torch.empty(f.shape, dtype=torch.int32,
                                      device=dev) for f in frames],
               "rms": [torch.empty_like(f) for f in frames]}
    # the deblending thresholds need the rms maps
    ctx.process_batch(frames, p, table=table, outputs=outputs,
                      write_rms=True)
    torch.cuda.synchronize()
    nsrc = table.count()
    sp = SubtractParams()
    coef = torch.from_numpy(_sub_coef(nfr, sp)).to(dev).contiguous()

    def timed(fn, k):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    holder = {}

    def deblend():
        holder["db"] = ctx.deblend(frames, outputs["bkg"], outputs["rms"],
                                   outputs["labels"], table, p)

    def auto():
        mom = ctx.source_moments(frames, outputs["bkg"], outputs["labels"],
                                 table)
        holder["mom"] = mom
        holder["auto"] = ctx.photometry_auto(frames, outputs["bkg"], table,
                                             mom)

    def subtract():
        ctx.subtract(frames, templates, sp, coef)

    log(f"timing {args.steps} steps of each")
    ms_db = timed(deblend, args.steps)
    nobj = holder["db"]["table"].count()
    db_diag = holder["db"]["diag"].cpu().tolist()
    ms_auto = timed(auto, args.steps)
    ms_sub = timed(subtract, args.steps)
    ctx.profile(True)
    for _ in range(2):
        deblend()
        auto()
        subtract()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    kern = {k: v0 / v1 for k, (v0, v1) in prof.items()}
    kw = 2 * sp.half_width + 1
    sub_flops = 2.0 * kw * kw * npx            # one FMA per tap and pixel
    ks = kern.get("k_subtract")
    roof = None
    if ks:
        tfs = sub_flops / (ks * 1e-3) / 1e12
        roof = {"kernel": "k_subtract", "bound": "alu",
                "achieved": round(tfs, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s",
                "frac": round(tfs / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": measured_traffic("k_subtract", "next16"),
                "algo_flops_per_launch": sub_flops,
                "ms_per_launch": round(ks, 4)}
    # deblending: each of the nthresh levels reads the candidates' pixel
    # values once and the object map is written once (4 B each)
    npix_c = int(table.cols["npix"][:nsrc].sum().item())
    nthr = ipp.DeblendParams().nthresh
    db_bytes = 4.0 * npix_c * (nthr + 1)
    kdb = sum(kern.get(k, 0.0) for k in ("k_db_small", "k_db_large",
                                          "k_db_write"))
    roof_db = None
    if kdb:
        gbs = db_bytes / (kdb * 1e-3) / 1e9
        roof_db = {"kernel": "k_db_small + k_db_large + k_db_write",
                   "bound": "hbm", "achieved": round(gbs, 1),
                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                   "algo_bytes_per_launch": db_bytes,
                   "candidate_pixels": npix_c, "levels": nthr,
                   "ms_per_launch": round(kdb, 4)}
    roof_kron = None
    kk = kern.get("k_kron", 0.0) + kern.get("k_kron_big", 0.0)
    if kk:
        kf = kron_flops(holder["mom"][:nsrc].cpu().numpy(),
                        holder["auto"]["kron_radius"][:nsrc].cpu().numpy())
        tfs = kf / (kk * 1e-3) / 1e12
        roof_kron = {"kernel": "k_kron + k_kron_big", "bound": "alu",
                     "achieved": round(tfs, 4),
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tfs / FP64_VECTOR_PEAK_TFLOPS, 5),
                     "traffic": measured_traffic("k_kron", "next16"),
                     "algo_flops_per_launch": kf,
                     "ms_per_launch": round(kk, 4)}
    res = {
        "metric": "Mpix/s of the stamp convolution and difference image",
        "value": round(npx / 1e6 / (ms_sub * 1e-3), 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_sub, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": SUB_DESC, "name": "next16", "frames": nfr,
                   "kernel": [kw, kw], "stamp": sp.stamp,
                   "basis": {"sigmas": list(sp.sigmas),
                             "orders": list(sp.orders)},
                   "spatial_order": sp.spatial_order,
                   "bkg_order": sp.bkg_order},
        "roofline": roof,
        "deblend": {"workload": "deblending and cleaning of the candidates "
                                "of the 16-frame stack (" + desc + ")",
                    "ms_per_step": round(ms_db, 4),
                    "mpix_per_s": round(npx / 1e6 / (ms_db * 1e-3), 1),
                    "candidates": nsrc, "objects": nobj,
                    "diag": db_diag,
                    "candidates_per_s": round(nsrc / (ms_db * 1e-3), 1),
                    "roofline": roof_db},
        "auto_photometry": {"workload": "second moments and AUTO (Kron) "
                                        "photometry of the candidates",
                            "ms_per_step": round(ms_auto, 4),
                            "sources": nsrc,
                            "sources_per_s": round(nsrc / (ms_auto * 1e-3),
                                                   1),
                            "roofline": roof_kron},
        "kernels_ms": {k: round(v, 4) for k, v in
                       sorted(kern.items(), key=lambda kv: -kv[1])},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def calibration_copy(mib, dev):
    """One device-to-device copy of `mib` MiB: a kernel of known traffic
    that scales the HBM byte counters of a profiled run."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def run_gray(args):
    """Gray-scale transformations of the 16-frame stack (Sec. 2.2.6): the
    zscale range of every frame and a logarithmic map over it, and histogram
    equalization (4096 bins)."""
    import torch
    import paper_2502_10783_amd as ipp

    dev = torch.device("cuda:0")
    nfr, desc = WORKLOADS["stack16"]
    if args.frames:
        nfr = min(nfr, args.frames)
    log(f"generating {nfr} frames of stack16 on the GPU")
    frames = make_frames("stack16", nfr, dev)
    if args.calib_copy:
        calibration_copy(args.calib_copy, dev)
    ctx = ipp.Context(0)
    out_map = [torch.empty_like(f) for f in frames]
    out_eq = [torch.empty_like(f) for f in frames]

    def zmap():
        z = ctx.zscale(frames)
        ctx.gray_map(frames, ipp.IPP_MAP_LOG, z, 1000.0, out=out_map)

    def equalize():
        ctx.equalize(frames, nbins=4096, out=out_eq)

    def timed(fn, k):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    log(f"timing {args.steps} steps of each")
    ms_map = timed(zmap, args.steps)
    ms_eq = timed(equalize, args.steps)
    ctx.profile(True)
    for _ in range(3):
        zmap()
        equalize()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    kern = {k: v0 / v1 for k, (v0, v1) in prof.items()}
    npx = sum(f.numel() for f in frames)
    # algorithmic bytes per pixel of each pass
    per_px = {"k_gray_map": 8, "k_eq_map": 8, "k_eq_hist": 4,
              "k_eq_minmax": 4}

    def hbm(k):
        gbs = per_px[k] * npx / (kern[k] * 1e-3) / 1e9
        return {"kernel": k, "bound": "hbm", "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "algo_bytes_per_launch": per_px[k] * npx,
                "ms_per_launch": round(kern[k], 4)}

    dom = max(per_px, key=lambda k: kern.get(k, 0.0))
    res = {
        "metric": "Mpix/s, zscale range + logarithmic map of every frame",
        "value": round(npx / 1e6 / (ms_map * 1e-3), 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_map, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc if nfr == WORKLOADS["stack16"][0] else
                   f"first {nfr} frames of: {desc}", "name": "gray16",
                   "frames": nfr, "map": "log", "a": 1000.0,
                   "zscale_samples": 1000, "contrast": 0.25,
                   "equalize_bins": 4096},
        "map_GBps": round(8 * npx / (ms_map * 1e-3) / 1e9, 1),
        "equalize": {"ms_per_step": round(ms_eq, 4),
                     "mpix_per_s": round(npx / 1e6 / (ms_eq * 1e-3), 1),
                     "GBps_at_16B_per_px": round(
                         16 * npx / (ms_eq * 1e-3) / 1e9, 1)},
        "roofline": dict(hbm(dom), traffic=measured_traffic(dom, "gray16")),
        "roofline_map": dict(hbm("k_gray_map"),
                             traffic=measured_traffic("k_gray_map",
                                                      "gray16")),
        "kernels_ms": {k: round(v, 4) for k, v in
                       sorted(kern.items(), key=lambda kv: -kv[1])},
    }
    print(json.dumps(res), flush=True)




def run_plain(ctx, frames, p, tables, refine):
    """Eager per-frame path: one background, detect, count, photometry (and
    refinement) call per frame; with the refinement the photometry is
    written by the refinement's first evaluation, as in the batched step."""
    from dataclasses import replace
    from paper_2502_10783_amd import _lib as L
    p_eager = replace(p, flags=p.flags | L.IPP_F_NO_GRAPH)
    n = 0
    for f, t in zip(frames, tables):
        bg = ctx.background([f], p)
        d = ctx.detect([f], bg["bkg"], bg["rms"], p, table=t)
        k = t.count()                             # host sync per frame
        n += k
        if not refine:
            ctx.photometry([f], bg["bkg"], d["table"], p)
        elif k:
            ctx.refine_centroids([f], bg["bkg"], t, p_eager,
                                 steps=REFINE_STEPS, r_c=REFINE_RC,
                                 use_count=True,
                                 x_out=t.extra_x, y_out=t.extra_y,
                                 write_photometry=True)
    return n


def flux_error_sample(frame_cpu, bkg_cpu, table_rows, params, k=64):
    """Max flux error of k sources of frame 0 against the oracle, on the
    GPU's own background map, in units of the flux's condition scale."""
    import numpy as np
    import oracle
    from oracle import photometry as oph
    sel = np.nonzero(table_rows["frame"] == 0)[0]
    sel = sel[np.linspace(0, sel.size - 1, min(k, sel.size)).astype(int)]
    ph = oph.photometry(frame_cpu.numpy(), bkg_cpu, table_rows["x"][sel],
                        table_rows["y"][sel], oracle.Params())
    raw = ph["flux"] + ph["sky"] * ph["area_ap"]
    scale = np.abs(raw) + ph["area_ap"] * np.abs(ph["sky"]) + 1e-30
    return float(np.max(np.abs(table_rows["flux_ap"][sel] - ph["flux"])
                        / scale))


def refine_error_sample(frame_cpu, bkg_cpu, table_rows, xr, yr, params,
                        k=4):
    """Max distance (px) between the refined centres of k sources of frame
    0 and the oracle's refinement of the same start positions."""
    import numpy as np
    import oracle
    from oracle.refine import refine_centroids
    sel = np.nonzero(table_rows["frame"] == 0)[0]
    sel = sel[np.linspace(0, sel.size - 1, min(k, sel.size)).astype(int)]
    xo, yo = refine_centroids(frame_cpu.numpy(), bkg_cpu,
                              table_rows["x"][sel], table_rows["y"][sel],
                              oracle.Params(), steps=REFINE_STEPS,
                              r_c=REFINE_RC)
    return float(np.max(np.hypot(xr[sel] - xo, yr[sel] - yo)))


def run_pipeline(workload, args, dev, quick=False):
    """Batched vs plain on one workload; returns its result dict (and the
    frames and outputs for the checks)."""
    import torch
    import paper_2502_10783_amd as ipp

    nfr, desc = WORKLOADS[workload]
    if args.frames:
        nfr = min(nfr, args.frames)
    refine = workload in REFINED
    log(f"[{workload}] generating {nfr} frames on the GPU")
    t0 = time.time()
    frames = make_frames(workload, nfr, dev)
    torch.cuda.synchronize()
    log(f"[{workload}] generated in {time.time() - t0:.1f} s")
    mpix = sum(f.numel() for f in frames) / 1e6
    npx = sum(f.numel() for f in frames)
    if args.calib_copy and not quick:
        calibration_copy(args.calib_copy, dev)
    p = ipp.Params()
    ctx = ipp.Context(0)
    tuned = None
    if workload == "uneven":
        log(f"[{workload}] autotuning mesh size and tile shape on the batch")
        t0 = time.time()
        p, tms = ctx.autotune(frames, p)
        tuned = {"mesh": p.mesh_h, "tile": [p.tile_h, p.tile_w],
                 "best_ms": round(tms, 4),
                 "tuning_s": round(time.time() - t0, 2)}
        log(f"[{workload}] autotuner: {tuned}")
    cap = npx // 64 + 4096
    table = ipp.SourceTable(cap, len(frames), dev)
    outputs = {"bkg": [torch.empty_like(f) for f in frames],
               "labels": [torch.empty(f.shape, dtype=torch.int32, device=dev)
                          for f in frames], "rms": None}
    xr = torch.empty(cap, dtype=torch.float64, device=dev)
    yr = torch.empty(cap, dtype=torch.float64, device=dev)

    # with the refinement, the photometry of every candidate is written by
    # the refinement's first evaluation (its sky is that evaluation's)
    # instead of a separate photometry launch
    def step():
        ctx.process_batch(frames, p, table=table, outputs=outputs,
                          photometry=not refine)
        if refine:
            ctx.refine_centroids(frames, outputs["bkg"], table, p,
                                 steps=REFINE_STEPS, r_c=REFINE_RC,
                                 use_count=True, x_out=xr, y_out=yr,
                                 write_photometry=True)

    steps = args.steps if not quick else max(3, args.steps)
    log(f"[{workload}] warmup")
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    nsrc = table.count()
    diag = outputs["diag"].cpu().tolist()
    if nsrc > cap or diag[2]:
        raise RuntimeError(f"capacity exceeded: sources {nsrc} > {cap} or "
                           f"records overflow {diag}")

    log(f"[{workload}] timing {steps} batched steps")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps

    ms_plain, psrc = None, 0
    plain_steps = args.plain_steps
    if plain_steps > 0:
        log(f"[{workload}] timing {plain_steps} plain per-frame steps")
        ptables = []
        for f in frames:
            t = ipp.SourceTable(f.numel() // 64 + 4096, 1, dev)
            if refine:
                t.extra_x = torch.empty(t.capacity, dtype=torch.float64,
                                        device=dev)
                t.extra_y = torch.empty_like(t.extra_x)
            ptables.append(t)
        run_plain(ctx, frames, p, ptables, refine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            psrc = run_plain(ctx, frames, p, ptables, refine)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) * 1e3 / plain_steps
        del ptables
        torch.cuda.empty_cache()

    log(f"[{workload}] per-kernel event timing")
    nprof = 2
    ctx.profile(True)
    for _ in range(nprof):
        step()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    kern = {k: {"ms_total": v[0] / nprof, "launches": v[1] // nprof,
                "ms_avg": v[0] / v[1]} for k, v in prof.items()}
    # algorithmic flops of the photometry launches of one step
    fl_fwd = aperture_flops_per_source(p.r_ap, p.r_in, p.r_out)
    fl_rc = aperture_flops_per_source(REFINE_RC, p.r_in, p.r_out)
    # (the refinement: per step a forward and a backward at r_c, all in
    # k_refine; the normaliser's aperture is taken in the first step's
    # evaluation over that step's sky, so it adds its own circle only)
    fl_norm = aperture_flops_per_source(p.r_ap, 0.0, 0.0)
    flops = {"k_aperture": nsrc * fl_fwd,
             "k_refine": (nsrc * (fl_norm + 2 * fl_rc * REFINE_STEPS)
                          if refine else 0.0)}
    dom = max(kern, key=lambda k: kern[k]["ms_total"])
    roof = roofline(kern, dom, npx, flops)
    roof["traffic"] = measured_traffic(dom, workload)
    hb = [k for k in kern if k in ALGO_BYTES_PER_PX]
    roof_hbm = None
    if hb:
        hk = max(hb, key=lambda k: kern[k]["ms_total"])
        roof_hbm = roofline(kern, hk, npx, flops)
        roof_hbm["traffic"] = measured_traffic(hk, workload)
    algo = step_algo_bytes(npx, nsrc, REFINE_STEPS if refine else 0)
    res = {
        "ms_per_step": round(ms, 4),
        "mpix_per_s": round(mpix / (ms * 1e-3), 2),
        "sources_per_step": nsrc,
        "sources_per_s": round(nsrc / (ms * 1e-3), 1),
        "plain": None if ms_plain is None else {
            "ms_per_step": round(ms_plain, 3),
            "mpix_per_s": round(mpix / (ms_plain * 1e-3), 2),
            "sources_per_s": round(psrc / (ms_plain * 1e-3), 1)},
        "speedup_vs_plain": (None if ms_plain is None
                             else round(ms_plain / ms, 3)),
        "step_hbm": {"algo_bytes": algo,
                     "achieved_GBps": round(algo / (ms * 1e-3) / 1e9, 1),
                     "frac": round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                   4)},
        "config": {"workload": desc if nfr == WORKLOADS[workload][0]
                   else f"first {nfr} frames of: {desc}", "name": workload,
                   "frames": len(frames), "mpix_per_step": round(mpix, 3),
                   "mesh": p.mesh_h, "tile": [p.tile_h or 64, p.tile_w or 64],
                   "autotuned": tuned, "det_nsigma": p.det_nsigma,
                   "min_area": p.min_area,
                   "aperture": [p.r_ap, p.r_in, p.r_out],
                   "refinement": ({"steps": REFINE_STEPS, "r_c": REFINE_RC,
                                   "eta": REFINE_ETA} if refine else None)},
        "kernels_ms_per_step": {k: round(v["ms_total"], 4) for k, v in
                                sorted(kern.items(),
                                       key=lambda kv: -kv[1]["ms_total"])},
        "roofline": roof,
        "roofline_hbm_kernel": roof_hbm,
    }
    if not quick:
        log(f"[{workload}] flux check against the oracle")
        rows = table.rows()
        b0 = outputs["bkg"][0].cpu().numpy()
        f0 = frames[0].cpu()
        res["flux_err_max"] = flux_error_sample(f0, b0, rows, p)
        if refine:
            res["refine_err_px_max"] = refine_error_sample(
                f0, b0, rows, xr[:nsrc].cpu().numpy(),
                yr[:nsrc].cpu().numpy(), p)
    ctx.close()
    del frames, outputs, table, xr, yr
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload",
                    choices=sorted(WORKLOADS) + ["grad64", "gray16",
                                                 "next16"],
                    default="crowded",
                    help="grad64: the forward + backward of the aperture "
                         "flux and of the asinh stretch; gray16: zscale, "
                         "point map and histogram equalization of the "
                         "16-frame stack; next16: deblending, AUTO "
                         "photometry and stamp subtraction of the 16-frame "
                         "stack (each its own metric)")
    ap.add_argument("--frames", type=int, default=0,
                    help="frames of the workload to use (0 = all)")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 16-frame and uneven-batch sub-results")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-core CPU leg (0 = the "
                         "host's cores, at most 16)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB "
                         "(a kernel of known traffic, to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single "
              "MI355X and has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "grad64":
        run_grad(args)
        return
    if args.workload == "gray16":
        run_gray(args)
        return
    if args.workload == "next16":
        run_next(args)
        return

    # the CPU leg first, in worker processes started before this process
    # touches the GPU
    cpu = None
    if not args.no_cpu:
        workers = args.cpu_workers or min(os.cpu_count() or 1, 16)
        log(f"oracle CPU baseline (1 core, then {workers} processes)")
        if args.workload == "crowded":
            cpu = cpu_baseline("crowded", 0.1, 40, workers)
        else:
            cpu = cpu_baseline(args.workload, 0.25, 0, workers)

    import torch
    dev = torch.device("cuda:0")
    main_res = run_pipeline(args.workload, args, dev)
    extra = {}
    if args.workload == "crowded" and not args.no_extra and not args.frames:
        for w in ("stack16", "uneven"):
            r = run_pipeline(w, args, dev, quick=True)
            extra[w] = {k: r[k] for k in
                        ("ms_per_step", "mpix_per_s", "sources_per_s",
                         "sources_per_step", "plain", "speedup_vs_plain",
                         "step_hbm", "config", "roofline")}
    ms = main_res["ms_per_step"]
    res = {
        "metric": METRIC,
        "value": main_res["mpix_per_s"],
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
    }
    res.update({k: v for k, v in main_res.items()
                if k not in ("ms_per_step", "mpix_per_s")})
    res["cpu_baseline"] = cpu
    if extra:
        res["other_configs"] = extra
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
