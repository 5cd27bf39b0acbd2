"""Python binding of libipp with torch tensors as device memory.

Marshals torch tensors into the C ABI of include/ipp.h; every computation
runs in libipp's HIP kernels on the tensors' GPU, asynchronously on the
current torch stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, fields
from typing import List, Optional, Sequence

import torch

from . import _lib as L


@dataclass
class Params:
    """Method parameters (ipp_params); defaults are the paper's settings."""
    mesh_h: int = 64
    mesh_w: int = 64
    filter_h: int = 3
    filter_w: int = 3
    clip_iters: int = 3
    estimator: int = L.IPP_EST_SEXTRACTOR
    clip_sigma: float = 3.0
    median_factor: float = 3.0
    mean_factor: float = 2.0
    min_valid: int = 100
    min_area: int = 5
    det_nsigma: float = 1.5
    connectivity: int = 8
    sky_clip_iters: int = 3
    sky_clip_sigma: float = 3.0
    r_ap: float = 5.0
    r_in: float = 8.0
    r_out: float = 12.0
    tile_h: int = 0
    tile_w: int = 0
    flags: int = 0

    def to_c(self) -> L.IppParams:
        c = L.IppParams()
        for f in fields(self):
            setattr(c, f.name, getattr(self, f.name))
        return c


@dataclass
class DeblendParams:
    """Deblending and cleaning parameters (ipp_deblend_params)."""
    nthresh: int = 32
    clean: int = 1
    mincont: float = 0.005
    clean_param: float = 1.0

    def to_c(self) -> L.IppDeblendParams:
        c = L.IppDeblendParams()
        for f in fields(self):
            setattr(c, f.name, getattr(self, f.name))
        return c


@dataclass
class SubtractParams:
    """Stamp convolution and subtraction parameters
    (ipp_subtract_params)."""
    half_width: int = 10
    stamp: int = 21
    sigmas: tuple = (0.7, 1.5, 3.0)
    orders: tuple = (6, 4, 2)
    spatial_order: int = 2
    bkg_order: int = 1

    def to_c(self) -> L.IppSubtractParams:
        c = L.IppSubtractParams()
        c.half_width, c.stamp = self.half_width, self.stamp
        c.n_gauss = len(self.sigmas)
        c.spatial_order, c.bkg_order = self.spatial_order, self.bkg_order
        for g, (s, o) in enumerate(zip(self.sigmas, self.orders)):
            c.sigma[g] = s
            c.order[g] = o
        return c


class IppError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.lib().ipp_status_string(status).decode()}"
                         f" ({status}): {msg}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_gpu_f32(t: torch.Tensor, what: str):
    if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2
            and t.stride(1) == 1):
        raise ValueError(f"{what}: need a 2-D float32 CUDA tensor with "
                         "unit column stride")


def _check_map(t: torch.Tensor, fr: torch.Tensor, what: str,
               dtype=torch.float32):
    """A per-pixel map of frame fr as the library reads it: dense h x w
    (row pitch w) of the given dtype on the GPU."""
    if not (t.is_cuda and t.dtype == dtype and t.dim() == 2
            and tuple(t.shape) == tuple(fr.shape) and t.is_contiguous()):
        raise ValueError(f"{what}: need a contiguous {dtype} CUDA tensor of "
                         f"the frame's shape {tuple(fr.shape)}")


def frames_c(frames: Sequence[torch.Tensor], masks=None):
    arr = (L.IppFrame * len(frames))()
    for i, fr in enumerate(frames):
        _check_gpu_f32(fr, f"frame {i}")
        arr[i].pix = fr.data_ptr()
        mk = masks[i] if masks is not None else None
        if mk is not None:
            # the library reads the mask with the frame's row pitch
            if not (mk.is_cuda and mk.dtype == torch.uint8 and mk.dim() == 2
                    and tuple(mk.shape) == tuple(fr.shape)
                    and mk.stride(1) == 1 and mk.stride(0) == fr.stride(0)):
                raise ValueError(f"mask {i}: need a uint8 CUDA tensor of the "
                                 "frame's shape and row pitch")
        arr[i].mask = mk.data_ptr() if mk is not None else None
        arr[i].pitch = fr.stride(0)
        arr[i].h, arr[i].w = fr.shape
    return arr


class SourceTable:
    """Struct-of-arrays source table in device memory."""

    DT = {"int32": torch.int32, "float64": torch.float64,
          "uint32": torch.int32}

    def __init__(self, capacity: int, n_frames: int, device):
        self.capacity = int(capacity)
        self.n_frames = n_frames
        self.cols = {name: torch.zeros(max(1, capacity), dtype=self.DT[dt],
                                       device=device)
                     for name, dt in L.SOURCE_COLUMNS}
        self.n_total = torch.zeros(1, dtype=torch.int64, device=device)
        self.frame_offsets = torch.zeros(n_frames + 1, dtype=torch.int64,
                                         device=device)

    def to_c(self, n_total=True) -> L.IppSources:
        s = L.IppSources()
        s.capacity = self.capacity
        s.n_total = self.n_total.data_ptr() if n_total else None
        s.frame_offsets = self.frame_offsets.data_ptr()
        for name, _ in L.SOURCE_COLUMNS:
            setattr(s, name, self.cols[name].data_ptr())
        return s

    def count(self) -> int:
        return int(self.n_total.item())

    def rows(self):
        """Host copy (numpy) of the filled rows."""
        n = min(self.count(), self.capacity)
        out = {k: v[:n].cpu().numpy() for k, v in self.cols.items()}
        out["flags"] = out["flags"].view("uint32")
        return out


class Context:
    """A libipp context on one GPU (owns the device workspace)."""

    def __init__(self, device: int = 0):
        self.lib = L.lib()
        self.device = device
        h = C.c_void_p()
        st = self.lib.ipp_ctx_create(C.byref(h), device)
        if st != L.IPP_OK:
            raise IppError(st, "ipp_ctx_create")
        self.h = h
        self.ws_bytes = 0

    def close(self):
        if self.h:
            self.lib.ipp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != L.IPP_OK:
            raise IppError(st, self.lib.ipp_last_error(self.h).decode())

    def profile(self, on: bool):
        """Start (clearing totals) or stop per-kernel event timing."""
        self._check(self.lib.ipp_ctx_profile(self.h, 1 if on else 0))

    def profile_read(self):
        """{kernel: (total_ms, launches)} since profiling was switched on."""
        n = self.lib.ipp_ctx_profile_read(self.h, 0, None, None, None)
        names = C.create_string_buffer(32 * max(n, 1))
        ms = (C.c_double * max(n, 1))()
        cnt = (C.c_int32 * max(n, 1))()
        self.lib.ipp_ctx_profile_read(self.h, n, names, ms, cnt)
        raw = names.raw
        return {raw[32 * i:32 * i + 32].split(b"\0")[0].decode():
                (ms[i], cnt[i]) for i in range(n)}

    def workspace_bytes(self, frames, params: Params, record_capacity=0):
        fc = frames_c(frames)
        pc = params.to_c()
        n = self.lib.ipp_workspace_bytes(fc, len(frames), C.byref(pc),
                                         int(record_capacity))
        if n == 0:
            raise IppError(L.IPP_E_INVALID_ARG, "ipp_workspace_bytes")
        return n

    def reserve(self, nbytes: int):
        self._check(self.lib.ipp_ctx_reserve(self.h, int(nbytes)))
        self.ws_bytes = max(self.ws_bytes, int(nbytes))

    def ensure(self, frames, params: Params, record_capacity=0):
        need = self.workspace_bytes(frames, params, record_capacity)
        if need > self.ws_bytes:
            self.reserve(need)

    # ---------------------------------------------------------- steps
    def background(self, frames: List[torch.Tensor], params: Params,
                   mesh: bool = False, masks=None):
        """Sec. 2.2.2: background and rms maps (and the meshes)."""
        self.ensure(frames, params)
        dev = frames[0].device
        n = len(frames)
        fc = frames_c(frames, masks)
        maps = (L.IppMaps * n)()
        out = {"bkg": [], "rms": []}
        meshes = (L.IppMesh * n)() if mesh else None
        if mesh:
            out.update({k: [] for k in ("bkg_raw", "rms_raw", "n_used",
                                        "bkg_mesh", "rms_mesh")})
        for i, fr in enumerate(frames):
            b = torch.empty_like(fr)
            r = torch.empty_like(fr)
            maps[i].bkg, maps[i].rms = b.data_ptr(), r.data_ptr()
            out["bkg"].append(b)
            out["rms"].append(r)
            if mesh:
                h, w = fr.shape
                ny = -(-h // params.mesh_h)
                nx = -(-w // params.mesh_w)
                t = {k: torch.empty((ny, nx), dtype=torch.float64, device=dev)
                     for k in ("bkg_raw", "rms_raw", "bkg_mesh", "rms_mesh")}
                t["n_used"] = torch.empty((ny, nx), dtype=torch.int32,
                                          device=dev)
                meshes[i].bkg_raw = t["bkg_raw"].data_ptr()
                meshes[i].rms_raw = t["rms_raw"].data_ptr()
                meshes[i].n_used = t["n_used"].data_ptr()
                meshes[i].bkg = t["bkg_mesh"].data_ptr()
                meshes[i].rms = t["rms_mesh"].data_ptr()
                for k, v in t.items():
                    out[k].append(v)
        flags = torch.zeros(n, dtype=torch.int32, device=dev)
        pc = params.to_c()
        self._check(self.lib.ipp_background(
            self.h, fc, n, C.byref(pc), maps, meshes, _ptr(flags),
            _stream()))
        out["flags"] = flags
        return out

    def detect(self, frames, bkg, rms, params: Params, capacity=None,
               table: Optional[SourceTable] = None):
        """Sec. 2.2.5: labels and source table against given maps."""
        self.ensure(frames, params)
        n = len(frames)
        dev = frames[0].device
        if table is None:
            if capacity is None:
                capacity = sum(f.numel() for f in frames) // 64 + 1024
            table = SourceTable(capacity, n, dev)
        maps = (L.IppMaps * n)()
        labels = []
        for i, fr in enumerate(frames):
            _check_map(bkg[i], fr, "bkg")
            _check_map(rms[i], fr, "rms")
            lab = torch.empty(fr.shape, dtype=torch.int32, device=dev)
            maps[i].bkg, maps[i].rms = bkg[i].data_ptr(), rms[i].data_ptr()
            maps[i].labels = lab.data_ptr()
            labels.append(lab)
        diag = torch.zeros(4, dtype=torch.int64, device=dev)
        src = table.to_c()
        pc = params.to_c()
        self._check(self.lib.ipp_detect(
            self.h, frames_c(frames), n, C.byref(pc), maps, C.byref(src),
            _ptr(diag), _stream()))
        return {"labels": labels, "table": table, "diag": diag}

    def photometry(self, frames, bkg, table: SourceTable, params: Params,
                   keep_sky=False, use_count=True):
        """Sec. 2.2.5: aperture photometry of the table rows."""
        n = len(frames)
        maps = (L.IppMaps * n)()
        for i in range(n):
            _check_map(bkg[i], frames[i], "bkg")
            maps[i].bkg = bkg[i].data_ptr()
        self.ensure(frames, params)
        lohi = None
        if keep_sky:
            lohi = torch.empty(2 * max(1, table.capacity),
                               dtype=torch.float64, device=frames[0].device)
        src = table.to_c(n_total=use_count)
        pc = params.to_c()
        self._check(self.lib.ipp_photometry(
            self.h, frames_c(frames), n, maps, C.byref(pc), C.byref(src),
            _ptr(lohi), _stream()))
        return lohi

    def photometry_backward(self, frames, bkg, table: SourceTable,
                            params: Params, sky_lohi, dL_dflux,
                            dpix=None, want_dxy=True, use_count=False):
        """Gradients of sum(dL_dflux * flux_ap): adds dL/dI into dpix
        (list of float32 maps, or None) and returns dL/d(x, y) (rows x 2)."""
        n = len(frames)
        maps = (L.IppMaps * n)()
        for i in range(n):
            _check_map(bkg[i], frames[i], "bkg")
            maps[i].bkg = bkg[i].data_ptr()
        dp = None
        if dpix is not None:
            dp = (C.c_void_p * n)()
            for i in range(n):
                if dpix[i] is not None:
                    _check_map(dpix[i], frames[i], "dpix")
                    dp[i] = dpix[i].data_ptr()
        dxy = None
        if want_dxy:
            dxy = torch.zeros((max(1, table.capacity), 2), dtype=torch.float64,
                              device=frames[0].device)
        g = dL_dflux.to(torch.float64).contiguous()
        src = table.to_c(n_total=use_count)
        pc = params.to_c()
        self._check(self.lib.ipp_photometry_backward(
            self.h, frames_c(frames), n, maps, C.byref(pc), C.byref(src),
            _ptr(sky_lohi), _ptr(g), dp, _ptr(dxy), _stream()))
        return dxy

    def refine_centroids(self, frames, bkg, table: SourceTable,
                         params: Params, steps: int = 10, eta: float = 3.0,
                         r_c: float = 2.0, x_out=None, y_out=None,
                         use_count=False, write_photometry=False):
        """Gradient-ascent centroid refinement of the table rows (frame, x,
        y) on the frames and their background maps: returns the refined
        (x, y) float64 tensors of `capacity` rows (x_out, y_out if given;
        they may be the table's own x and y columns).  write_photometry:
        the table's photometry columns at the starting centres are written
        too, from the first evaluation (as photometry() writes them)."""
        n = len(frames)
        maps = (L.IppMaps * n)()
        for i in range(n):
            _check_map(bkg[i], frames[i], "bkg")
            maps[i].bkg = bkg[i].data_ptr()
        fc = frames_c(frames)
        cap = max(1, table.capacity)
        need = self.lib.ipp_refine_workspace_bytes(fc, n, table.capacity)
        if need == 0:
            raise IppError(L.IPP_E_INVALID_ARG, "ipp_refine_workspace_bytes")
        if need > self.ws_bytes:
            self.reserve(need)
        dev = frames[0].device
        for t, what in ((x_out, "x_out"), (y_out, "y_out")):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64
                                      and t.is_contiguous()
                                      and t.numel() >= cap):
                raise ValueError(f"{what}: need a contiguous float64 CUDA "
                                 f"tensor of at least {cap} elements")
        if x_out is None:
            x_out = torch.empty(cap, dtype=torch.float64, device=dev)
        if y_out is None:
            y_out = torch.empty(cap, dtype=torch.float64, device=dev)
        src = table.to_c(n_total=use_count)
        pc = params.to_c()
        if write_photometry:
            pc.flags |= L.IPP_F_REFINE_PHOTOMETRY
        self._check(self.lib.ipp_refine_centroids(
            self.h, fc, n, maps, C.byref(pc), C.byref(src), float(r_c),
            float(eta), int(steps), _ptr(x_out), _ptr(y_out), _stream()))
        return x_out, y_out

    def asinh(self, v: torch.Tensor, a: float, b: float):
        """y = b * asinh(v / a) (float32, element-wise)."""
        if not (v.is_cuda and v.dtype == torch.float32):
            raise ValueError("v: need a float32 CUDA tensor")
        v = v.contiguous()
        y = torch.empty_like(v)
        self._check(self.lib.ipp_asinh(self.h, _ptr(v), _ptr(y), v.numel(),
                                       float(a), float(b), _stream()))
        return y

    def asinh_backward(self, v, dy, a: float, b: float, want_dv=True,
                       want_dab=True):
        """(dL/dv, tensor([dL/da, dL/db]))."""
        if not (v.is_cuda and dy.is_cuda and v.dtype == torch.float32
                and dy.dtype == torch.float32 and v.numel() == dy.numel()):
            raise ValueError("v, dy: need float32 CUDA tensors of one size")
        if want_dab and self.ws_bytes < (1 << 16):
            self.reserve(1 << 16)
        v = v.contiguous()
        dy = dy.contiguous()
        dv = torch.empty_like(v) if want_dv else None
        dab = (torch.zeros(2, dtype=torch.float64, device=v.device)
               if want_dab else None)
        self._check(self.lib.ipp_asinh_backward(
            self.h, _ptr(v), _ptr(dy), _ptr(dv), _ptr(dab), v.numel(),
            float(a), float(b), _stream()))
        return dv, dab

    @staticmethod
    def _ab(ab: torch.Tensor, v: torch.Tensor):
        if not (isinstance(ab, torch.Tensor) and ab.is_cuda
                and ab.dtype == torch.float64 and ab.numel() == 2
                and ab.is_contiguous() and ab.device == v.device):
            raise ValueError("ab: need a contiguous float64 CUDA tensor "
                             "(a, b) on v's device")
        return ab

    def asinh_dev(self, v: torch.Tensor, ab: torch.Tensor):
        """y = b * asinh(v / a) with (a, b) = ab read on the device."""
        if not (v.is_cuda and v.dtype == torch.float32):
            raise ValueError("v: need a float32 CUDA tensor")
        v = v.contiguous()
        y = torch.empty_like(v)
        self._check(self.lib.ipp_asinh_dev(
            self.h, _ptr(v), _ptr(y), v.numel(), _ptr(self._ab(ab, v)),
            _stream()))
        return y

    def asinh_backward_dev(self, v, dy, ab: torch.Tensor, want_dv=True,
                           want_dab=True):
        """(dL/dv, tensor([dL/da, dL/db])) with (a, b) = ab on the
        device."""
        if not (v.is_cuda and dy.is_cuda and v.dtype == torch.float32
                and dy.dtype == torch.float32 and v.numel() == dy.numel()):
            raise ValueError("v, dy: need float32 CUDA tensors of one size")
        if want_dab and self.ws_bytes < (1 << 16):
            self.reserve(1 << 16)
        v = v.contiguous()
        dy = dy.contiguous()
        dv = torch.empty_like(v) if want_dv else None
        dab = (torch.zeros(2, dtype=torch.float64, device=v.device)
               if want_dab else None)
        self._check(self.lib.ipp_asinh_backward_dev(
            self.h, _ptr(v), _ptr(dy), _ptr(dv), _ptr(dab), v.numel(),
            _ptr(self._ab(ab, v)), _stream()))
        return dv, dab

    def asinh_backward_noalloc(self, v, dy, a: float, b: float,
                               dv=None, dab=None):
        """ipp_asinh_backward_noalloc: the backward with its partials in the
        library's static scratch; writes into the given dv (float32, like
        v) and dab (float64 [2]) tensors, either may be None."""
        if not (v.is_cuda and dy.is_cuda and v.dtype == torch.float32
                and dy.dtype == torch.float32 and v.numel() == dy.numel()
                and v.is_contiguous() and dy.is_contiguous()):
            raise ValueError("v, dy: need contiguous float32 CUDA tensors of "
                             "one size")
        if dv is not None and not (dv.is_cuda and dv.dtype == torch.float32
                                   and dv.numel() == v.numel()
                                   and dv.is_contiguous()):
            raise ValueError("dv: need a contiguous float32 CUDA tensor "
                             "of v's size")
        if dab is not None and not (dab.is_cuda and dab.dtype ==
                                    torch.float64 and dab.numel() == 2):
            raise ValueError("dab: need a float64 CUDA tensor of 2 elements")
        self._check(self.lib.ipp_asinh_backward_noalloc(
            self.h, _ptr(v), _ptr(dy), _ptr(dv), _ptr(dab), v.numel(),
            float(a), float(b), _stream()))
        return dv, dab

    def deblend(self, frames, bkg, rms, labels, table: SourceTable,
                params: Params, dparams: Optional[DeblendParams] = None,
                capacity=None, scratch_bytes=None):
        """Sec. 2.2.5 deblending and cleaning of the detection's candidates
        (label maps and table): returns the object maps, the object table,
        each object's parent candidate label and the diagnostics.  The
        scratch pool grows (and the call is repeated) when a first try
        reports it too small."""
        n = len(frames)
        dev = frames[0].device
        dp = dparams or DeblendParams()
        npx = sum(f.numel() for f in frames)
        if capacity is None:
            capacity = 2 * max(table.capacity, 1) + 1024
        if scratch_bytes is None:
            scratch_bytes = 64 * npx + (1 << 20)
        fc = frames_c(frames)
        maps = (L.IppMaps * n)()
        objs = []
        for i, fr in enumerate(frames):
            _check_map(bkg[i], fr, "bkg")
            _check_map(rms[i], fr, "rms")
            _check_map(labels[i], fr, "labels", torch.int32)
            maps[i].bkg = bkg[i].data_ptr()
            maps[i].rms = rms[i].data_ptr()
            maps[i].labels = labels[i].data_ptr()
            objs.append(torch.empty(fr.shape, dtype=torch.int32, device=dev))
        optr = (C.c_void_p * n)(*[o.data_ptr() for o in objs])
        obj = SourceTable(capacity, n, dev)
        parent = torch.zeros(max(1, capacity), dtype=torch.int32, device=dev)
        diag = torch.zeros(4, dtype=torch.int64, device=dev)
        pc = params.to_c()
        dpc = dp.to_c()
        for _ in range(3):
            need = self.lib.ipp_deblend_workspace_bytes(
                fc, n, table.capacity, int(scratch_bytes))
            if need == 0:
                raise IppError(L.IPP_E_INVALID_ARG,
                               "ipp_deblend_workspace_bytes")
            if need > self.ws_bytes:
                self.reserve(need)
            cand = table.to_c()
            oc = obj.to_c()
            self._check(self.lib.ipp_deblend(
                self.h, fc, n, C.byref(pc), C.byref(dpc), maps,
                C.byref(cand), optr, C.byref(oc), _ptr(parent), _ptr(diag),
                _stream()))
            d = diag.cpu().tolist()
            if not (d[2] & 1):
                break
            scratch_bytes = int(d[0]) + (1 << 20)
        return {"objects": objs, "table": obj, "parent": parent,
                "diag": diag}

    def photometry_auto(self, frames, bkg, table: SourceTable,
                        moments: torch.Tensor, kron_factor=2.5, kron_min=3.5,
                        search=6.0, use_count=True):
        """AUTO (Kron) photometry of the table rows (frame, x, y) with their
        second moments (rows x 6, as source_moments returns): dict of
        float64 kron radius, flux, area and int32 flags per row."""
        n = len(frames)
        maps = (L.IppMaps * n)()
        for i in range(n):
            _check_map(bkg[i], frames[i], "bkg")
            maps[i].bkg = bkg[i].data_ptr()
        cap = max(1, table.capacity)
        if not (moments.is_cuda and moments.dtype == torch.float64 and
                moments.is_contiguous() and moments.dim() == 2 and
                moments.shape[1] == 6):
            raise ValueError("moments: need a contiguous float64 CUDA "
                             "tensor of rows x 6")
        mom = moments
        if mom.shape[0] < cap:
            mom = torch.full((cap, 6), float("nan"), dtype=torch.float64,
                             device=moments.device)
            mom[:moments.shape[0]] = moments
        self.ensure(frames, Params())
        dev = frames[0].device
        out = {k: torch.empty(cap, dtype=torch.float64, device=dev)
               for k in ("kron_radius", "flux", "area")}
        out["flags"] = torch.empty(cap, dtype=torch.int32, device=dev)
        ap = L.IppAutoParams(float(kron_factor), float(kron_min),
                             float(search))
        src = table.to_c(n_total=use_count)
        self._check(self.lib.ipp_photometry_auto(
            self.h, frames_c(frames), n, maps, C.byref(src), _ptr(mom),
            C.byref(ap), _ptr(out["kron_radius"]), _ptr(out["flux"]),
            _ptr(out["area"]), _ptr(out["flags"]), _stream()))
        return out

    def subtract(self, frames, templates, sp: SubtractParams, coef):
        """Sec. 2.2.4: difference images D = (I + B) - R (x) K of each frame
        I against its aligned template R; coef: float64 tensor [n, count]
        of the kernel and background polynomial coefficients."""
        n = len(frames)
        spc = sp.to_c()
        per = self.lib.ipp_subtract_coef_count(C.byref(spc))
        if per == 0:
            raise IppError(L.IPP_E_INVALID_ARG, "invalid subtract params")
        if not (coef.is_cuda and coef.dtype == torch.float64 and
                coef.is_contiguous() and coef.numel() == n * per):
            raise ValueError(f"coef: need a contiguous float64 CUDA tensor "
                             f"of {n} x {per} coefficients")
        for i in range(n):
            _check_gpu_f32(templates[i], f"template {i}")
        if self.ws_bytes < 4096 + 64 * n:
            self.reserve(4096 + 64 * n)
        out = [torch.empty(f.shape, dtype=torch.float32, device=f.device)
               for f in frames]
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in out])
        self._check(self.lib.ipp_subtract(
            self.h, frames_c(frames), frames_c(templates), n, C.byref(spc),
            _ptr(coef), ptrs, _stream()))
        return out

    def source_moments(self, frames, bkg, labels, table: SourceTable):
        """Second-order moments per table row: float64 tensor [rows, 6]
        (x2, y2, xy, a, b, theta)."""
        n = len(frames)
        self.ensure(frames, Params())
        maps = (L.IppMaps * n)()
        for i in range(n):
            _check_map(bkg[i], frames[i], "bkg")
            _check_map(labels[i], frames[i], "labels", torch.int32)
            maps[i].bkg = bkg[i].data_ptr()
            maps[i].labels = labels[i].data_ptr()
        cap = max(1, table.capacity)
        mom = torch.full((cap, 6), float("nan"), dtype=torch.float64,
                         device=frames[0].device)
        src = table.to_c()
        self._check(self.lib.ipp_source_moments(
            self.h, frames_c(frames), n, maps, C.byref(src), _ptr(mom),
            _stream()))
        return mom[:min(table.count(), table.capacity)]

    # ------------------------------------------------ gray scale (2.2.6)
    def _gray_reserve(self, n, nbins=0):
        need = self.lib.ipp_gray_workspace_bytes(n, nbins)
        if need == 0:
            raise IppError(L.IPP_E_INVALID_ARG, "ipp_gray_workspace_bytes")
        if need > self.ws_bytes:
            self.reserve(need)

    def zscale(self, frames, nsamples=1000, contrast=0.25, info=False):
        """zscale display range per frame: tensor [n, 2] (z1, z2), and with
        info=True also [n, 4] (samples, kept, fits, slope)."""
        n = len(frames)
        self._gray_reserve(n)
        dev = frames[0].device
        z = torch.zeros((n, 2), dtype=torch.float64, device=dev)
        inf = (torch.zeros((n, 4), dtype=torch.float64, device=dev)
               if info else None)
        self._check(self.lib.ipp_zscale(
            self.h, frames_c(frames), n, int(nsamples), float(contrast),
            _ptr(z), _ptr(inf), _stream()))
        return (z, inf) if info else z

    def gray_map(self, frames, kind: int, lohi: torch.Tensor, a=1000.0,
                 out=None):
        """Point map (IPP_MAP_*) of each frame over lohi[f] = (lo, hi)."""
        n = len(frames)
        self._gray_reserve(n)
        if lohi.dtype != torch.float64 or not lohi.is_contiguous():
            raise ValueError("lohi must be a contiguous float64 tensor")
        if out is None:
            out = [torch.empty(f.shape, dtype=torch.float32, device=f.device)
                   for f in frames]
        for i in range(n):
            _check_map(out[i], frames[i], "out")
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in out])
        self._check(self.lib.ipp_gray_map(
            self.h, frames_c(frames), n, int(kind), float(a), _ptr(lohi),
            ptrs, _stream()))
        return out

    def equalize(self, frames, nbins=4096, counts=False, out=None):
        """Histogram equalization of each frame (and, with counts=True, the
        histograms as an int32 tensor [n, nbins] holding uint32 counts)."""
        n = len(frames)
        self._gray_reserve(n, nbins)
        dev = frames[0].device
        if out is None:
            out = [torch.empty(f.shape, dtype=torch.float32, device=dev)
                   for f in frames]
        cnt = (torch.empty((n, nbins), dtype=torch.int32, device=dev)
               if counts else None)
        for i in range(n):
            _check_map(out[i], frames[i], "out")
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in out])
        self._check(self.lib.ipp_equalize(
            self.h, frames_c(frames), n, int(nbins), ptrs, _ptr(cnt),
            _stream()))
        return (out, cnt) if counts else out

    def autotune(self, frames, params: Params, mesh=True, tile=True,
                 cache_path: Optional[str] = None):
        """Fastest mesh size / tile shape for this batch on this device:
        returns (Params, ms)."""
        what = (L.IPP_TUNE_MESH if mesh else 0) | (L.IPP_TUNE_TILE if tile
                                                   else 0)
        pc = params.to_c()
        ms = C.c_double(0.0)
        self._check(self.lib.ipp_autotune(
            self.h, frames_c(frames), len(frames), C.byref(pc), what,
            cache_path.encode() if cache_path else None, C.byref(ms),
            _stream()))
        self.ws_bytes = max(self.ws_bytes, self.workspace_bytes(
            frames, params))
        out = Params(**{f.name: getattr(params, f.name)
                        for f in fields(params)})
        out.mesh_h, out.mesh_w = pc.mesh_h, pc.mesh_w
        out.tile_h, out.tile_w = pc.tile_h, pc.tile_w
        return out, ms.value

    def process_batch(self, frames, params: Params, capacity=None,
                      table: Optional[SourceTable] = None, outputs=None,
                      write_rms=False, masks=None, photometry=True):
        """Pipeline mode (Sec. 2.1): the whole path for a batch (masks:
        optional uint8 tensors, non-zero = pixel left out of the
        background statistics).  photometry=False stops after the source
        table (the photometry columns then come from photometry() or from
        refine_centroids(write_photometry=True))."""
        self.ensure(frames, params)
        n = len(frames)
        dev = frames[0].device
        if table is None:
            if capacity is None:
                capacity = sum(f.numel() for f in frames) // 64 + 1024
            table = SourceTable(capacity, n, dev)
        if outputs is None:
            outputs = {"bkg": [torch.empty_like(f) for f in frames],
                       "labels": [torch.empty(f.shape, dtype=torch.int32,
                                              device=dev) for f in frames],
                       "rms": ([torch.empty_like(f) for f in frames]
                               if write_rms else None)}
        maps = (L.IppMaps * n)()
        for i in range(n):
            _check_map(outputs["bkg"][i], frames[i], "bkg")
            _check_map(outputs["labels"][i], frames[i], "labels",
                       torch.int32)
            if write_rms:
                _check_map(outputs["rms"][i], frames[i], "rms")
            maps[i].bkg = outputs["bkg"][i].data_ptr()
            maps[i].labels = outputs["labels"][i].data_ptr()
            if write_rms:
                maps[i].rms = outputs["rms"][i].data_ptr()
        p = Params(**{f.name: getattr(params, f.name) for f in fields(params)})
        if write_rms:
            p.flags |= L.IPP_F_WRITE_RMS
        if not photometry:
            p.flags |= L.IPP_F_NO_PHOTOMETRY
        # frame flags and diagnostics are overwritten by every call: reuse
        # the caller's buffers so repeated calls keep the same device
        # addresses (they are part of the captured graph's signature)
        flags = outputs.get("flags")
        if not (isinstance(flags, torch.Tensor) and flags.numel() == n
                and flags.dtype == torch.int32 and flags.device == dev):
            flags = torch.zeros(n, dtype=torch.int32, device=dev)
        diag = outputs.get("diag")
        if not (isinstance(diag, torch.Tensor) and diag.numel() == 4
                and diag.dtype == torch.int64 and diag.device == dev):
            diag = torch.zeros(4, dtype=torch.int64, device=dev)
        src = table.to_c()
        pc = p.to_c()
        self._check(self.lib.ipp_process_batch(
            self.h, frames_c(frames, masks), n, C.byref(pc), maps,
            C.byref(src),
            _ptr(flags), _ptr(diag), _stream()))
        outputs.update({"table": table, "flags": flags, "diag": diag})
        return outputs
