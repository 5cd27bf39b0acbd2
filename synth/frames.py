"""Frame recipes for the five workloads and a torch renderer for them.

Workloads (rows x columns, float32 ADU, gain 1 e-/ADU):

* ``single``   1 frame 1024x1024; sky 1000 + 0.5 ADU/px along x; Poisson +
  Gaussian read noise sigma 10; 200 Gaussian stars, FWHM 3 px, flux
  log-uniform in [1e3, 1e6].
* ``stack16``  16 frames 4096x4096; sky 800 + 2nd-order polynomial + 50 ADU
  sinusoid of period 700 px; Poisson + read noise sigma 8; 5000 Moffat stars
  (beta 3, FWHM U(2, 5), flux log-U[5e2, 1e6]); cosmic rays on 1e-4 of the
  pixels (+U(5e3, 5e4) ADU); 2 dead columns.
* ``uneven``   256 frames drawn from {512x512, 1024x1024, 2048x4096,
  4096x4096}; star density log-U[1e-5, 5e-3] per px; flat sky U(200, 5000).
* ``grad64``   64 frames 2048x2048; sky as ``single``; 2000 Gaussian stars
  with FWHM U(2.5, 4); centroid guesses perturbed by N(0, 0.3 px).
* ``crowded``  32 frames 10560x10560; 1500 ADU + 1/f^2 Gaussian random field
  (rms 100); 100k Moffat stars (beta 2.5, FWHM U(2, 6), flux
  log-U[3e2, 3e6]); saturation at 65535.

Everything is generated in float64 and cast to float32 last.  A ``scale``
argument shrinks a recipe (rows, columns and star count) for tests that must
finish in seconds while keeping the same sky, noise and source mix.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import torch

SEED_BASE = 250210783
CONFIG_NAMES = ("single", "stack16", "uneven", "grad64", "crowded")
_UNEVEN_SIZES = ((512, 512), (1024, 1024), (2048, 4096), (4096, 4096))
_N_FRAMES = {"single": 1, "stack16": 16, "uneven": 256, "grad64": 64,
             "crowded": 32}


@dataclass
class FrameSpec:
    h: int
    w: int
    sky: str = "gradient"          # gradient | poly_sin | flat | grf
    sky_level: float = 1000.0
    sky_slope: float = 0.5
    sin_amp: float = 50.0
    sin_period: float = 700.0
    grf_rms: float = 100.0
    psf: str = "gauss"             # gauss | moffat
    beta: float = 3.0
    fwhm: tuple = (3.0, 3.0)
    flux: tuple = (1e3, 1e6)
    n_stars: int = 200
    read_sigma: float = 10.0
    poisson: bool = True
    cr_fraction: float = 0.0
    cr_range: tuple = (5e3, 5e4)
    dead_cols: int = 0
    saturate: Optional[float] = None
    centroid_jitter: float = 0.0
    extra: dict = field(default_factory=dict)


def _generator(config: str, frame: int, device) -> torch.Generator:
    cid = CONFIG_NAMES.index(config) if config in CONFIG_NAMES else 99
    g = torch.Generator(device=device)
    g.manual_seed((SEED_BASE * 1000003 + cid * 7919 + frame * 104729)
                  % (2 ** 62))
    return g


def _u(g, n, lo, hi, device):
    return lo + (hi - lo) * torch.rand(n, generator=g, device=device,
                                       dtype=torch.float64)


def _logu(g, n, lo, hi, device):
    return torch.exp(_u(g, n, math.log(lo), math.log(hi), device))


def config_frame_specs(config: str, scale: float = 1.0,
                       n_frames: Optional[int] = None):
    """The list of per-frame recipes of a workload (sizes drawn, seeded)."""
    n = _N_FRAMES[config] if n_frames is None else n_frames
    return [spec_for(config, i, scale) for i in range(n)]


def spec_for(config: str, frame: int, scale: float = 1.0) -> FrameSpec:
    """Recipe of one frame of a workload; ``scale`` shrinks it linearly."""
    def sz(v):
        return max(8, int(round(v * scale)))

    if config == "single":
        s = FrameSpec(h=sz(1024), w=sz(1024), sky="gradient", sky_level=1000.0,
                      sky_slope=0.5, psf="gauss", fwhm=(3.0, 3.0),
                      flux=(1e3, 1e6), n_stars=200, read_sigma=10.0)
    elif config == "stack16":
        s = FrameSpec(h=sz(4096), w=sz(4096), sky="poly_sin", sky_level=800.0,
                      psf="moffat", beta=3.0, fwhm=(2.0, 5.0),
                      flux=(5e2, 1e6), n_stars=5000, read_sigma=8.0,
                      cr_fraction=1e-4, dead_cols=2)
    elif config == "uneven":
        g = _generator(config, -1, "cpu")
        idx = torch.randint(0, 4, (_N_FRAMES[config],), generator=g)
        dens = torch.exp(math.log(1e-5) + (math.log(5e-3) - math.log(1e-5))
                         * torch.rand(_N_FRAMES[config], generator=g,
                                      dtype=torch.float64))
        sky = 200.0 + 4800.0 * torch.rand(_N_FRAMES[config], generator=g,
                                          dtype=torch.float64)
        k = frame % _N_FRAMES[config]
        h, w = _UNEVEN_SIZES[int(idx[k])]
        s = FrameSpec(h=sz(h), w=sz(w), sky="flat", sky_level=float(sky[k]),
                      psf="moffat", beta=3.0, fwhm=(2.0, 5.0),
                      flux=(5e2, 1e6), n_stars=0, read_sigma=8.0)
        s.n_stars = int(round(float(dens[k]) * s.h * s.w))
        return s
    elif config == "grad64":
        s = FrameSpec(h=sz(2048), w=sz(2048), sky="gradient",
                      sky_level=1000.0, sky_slope=0.5, psf="gauss",
                      fwhm=(2.5, 4.0), flux=(1e3, 1e6), n_stars=2000,
                      read_sigma=10.0, centroid_jitter=0.3)
    elif config == "crowded":
        s = FrameSpec(h=sz(10560), w=sz(10560), sky="grf", sky_level=1500.0,
                      grf_rms=100.0, psf="moffat", beta=2.5, fwhm=(2.0, 6.0),
                      flux=(3e2, 3e6), n_stars=100000, read_sigma=10.0,
                      saturate=65535.0)
    else:
        raise ValueError(f"unknown workload {config!r}")
    if scale != 1.0:
        s.n_stars = max(1, int(round(s.n_stars * scale * scale)))
    return s


def _sky(spec: FrameSpec, g, device):
    h, w = spec.h, spec.w
    x = torch.arange(w, device=device, dtype=torch.float64)[None, :]
    y = torch.arange(h, device=device, dtype=torch.float64)[:, None]
    if spec.sky == "flat":
        return torch.full((h, w), spec.sky_level, device=device,
                          dtype=torch.float64)
    if spec.sky == "gradient":
        return (spec.sky_level + spec.sky_slope * x).expand(h, w).clone()
    if spec.sky == "poly_sin":
        a = _u(g, 5, -40.0, 40.0, device)
        th = float(_u(g, 1, 0.0, 2 * math.pi, device))
        ph = float(_u(g, 1, 0.0, 2 * math.pi, device))
        u = 2.0 * x / max(w - 1, 1) - 1.0
        v = 2.0 * y / max(h - 1, 1) - 1.0
        poly = a[0] * u + a[1] * v + a[2] * u * u + a[3] * u * v + a[4] * v * v
        wave = spec.sin_amp * torch.sin(
            2 * math.pi * (x * math.cos(th) + y * math.sin(th))
            / spec.sin_period + ph)
        return spec.sky_level + poly + wave
    if spec.sky == "grf":
        noise = torch.randn((h, w), generator=g, device=device,
                            dtype=torch.float64)
        fk = torch.fft.rfft2(noise)
        ky = torch.fft.fftfreq(h, device=device, dtype=torch.float64)[:, None]
        kx = torch.fft.rfftfreq(w, device=device, dtype=torch.float64)[None, :]
        k2 = kx * kx + ky * ky
        amp = torch.where(k2 > 0, 1.0 / torch.sqrt(k2.clamp_min(1e-30)),
                          torch.zeros_like(k2))        # P(k) ~ k^-2
        field = torch.fft.irfft2(fk * amp, s=(h, w))
        field = field - field.mean()
        field = field * (spec.grf_rms / field.std().clamp_min(1e-30))
        return spec.sky_level + field
    raise ValueError(spec.sky)


def _stars(spec: FrameSpec, g, device):
    n = spec.n_stars
    xs = _u(g, n, -0.5, spec.w - 0.5, device)
    ys = _u(g, n, -0.5, spec.h - 0.5, device)
    fl = _logu(g, n, spec.flux[0], spec.flux[1], device)
    fw = _u(g, n, spec.fwhm[0], spec.fwhm[1], device)
    return xs, ys, fl, fw


def _render_stars(img, spec, xs, ys, fl, fw, chunk=4096):
    h, w = spec.h, spec.w
    if xs.numel() == 0:
        return
    half = int(math.ceil(5.0 * spec.fwhm[1]))
    if spec.psf == "moffat":
        half = int(math.ceil(6.0 * spec.fwhm[1]))
    d = torch.arange(-half, half + 1, device=img.device, dtype=torch.float64)
    flat = img.view(-1)
    for s in range(0, xs.numel(), chunk):
        x, y = xs[s:s + chunk, None], ys[s:s + chunk, None]
        f, fwhm = fl[s:s + chunk, None], fw[s:s + chunk, None]
        px = torch.round(x) + d[None, :]             # (n, k) pixel columns
        py = torch.round(y) + d[None, :]
        if spec.psf == "gauss":
            sig = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
            c = 1.0 / (sig * math.sqrt(2.0))
            gx = 0.5 * (torch.erf((px + 0.5 - x) * c)
                        - torch.erf((px - 0.5 - x) * c))
            gy = 0.5 * (torch.erf((py + 0.5 - y) * c)
                        - torch.erf((py - 0.5 - y) * c))
            val = f[:, :, None] * gy[:, :, None] * gx[:, None, :]
        else:
            beta = spec.beta
            alpha = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
            r2 = ((px - x)[:, None, :] ** 2 + (py - y)[:, :, None] ** 2)
            a2 = (alpha * alpha)[:, :, None]
            val = (f[:, :, None] * (beta - 1.0) / (math.pi * a2)
                   * (1.0 + r2 / a2) ** (-beta))
            val = torch.where(r2 <= float(half * half), val,
                              torch.zeros_like(val))
        ix = px.long()[:, None, :].expand_as(val)
        iy = py.long()[:, :, None].expand_as(val)
        ok = (ix >= 0) & (ix < w) & (iy >= 0) & (iy < h)
        flat.index_add_(0, (iy * w + ix)[ok], val[ok])


def render(spec: FrameSpec, config: str, frame: int, device="cpu"):
    """Render one frame; returns (float32 frame [h, w], truth dict)."""
    g = _generator(config, frame, device)
    img = _sky(spec, g, device)
    xs, ys, fl, fw = _stars(spec, g, device)
    _render_stars(img, spec, xs, ys, fl, fw)
    if spec.poisson:
        img = torch.poisson(img.clamp_min(0.0), generator=g)
    if spec.read_sigma > 0:
        img = img + spec.read_sigma * torch.randn(
            img.shape, generator=g, device=device, dtype=torch.float64)
    if spec.cr_fraction > 0:
        ncr = int(round(spec.cr_fraction * spec.h * spec.w))
        idx = torch.randint(0, spec.h * spec.w, (ncr,), generator=g,
                            device=device)
        img.view(-1).index_add_(0, idx, _u(g, ncr, spec.cr_range[0],
                                           spec.cr_range[1], device))
    if spec.dead_cols > 0:
        cols = torch.randint(0, spec.w, (spec.dead_cols,), generator=g,
                             device=device)
        img[:, cols] = 0.0
    if spec.saturate is not None:
        img = img.clamp_max(spec.saturate)
    truth = {"x": xs, "y": ys, "flux": fl, "fwhm": fw}
    if spec.centroid_jitter > 0:
        truth["x_guess"] = xs + spec.centroid_jitter * torch.randn(
            xs.shape, generator=g, device=device, dtype=torch.float64)
        truth["y_guess"] = ys + spec.centroid_jitter * torch.randn(
            ys.shape, generator=g, device=device, dtype=torch.float64)
    return img.to(torch.float32).contiguous(), truth


def make_frame(config: str, frame: int = 0, scale: float = 1.0,
               device="cpu", **overrides):
    """Recipe + render in one call; ``overrides`` replace recipe fields."""
    spec = spec_for(config, frame, scale)
    if overrides:
        spec = replace(spec, **overrides)
    img, truth = render(spec, config, frame, device)
    return img, truth, spec
