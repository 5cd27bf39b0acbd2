"""Method parameters of the oracle (plain dataclass; defaults = the paper's)."""
from dataclasses import dataclass

# Background estimators, Eq. 1-4 of Sec. 2.2.2.
EST_SEXTRACTOR = 0   # Eq. 3: 2.5 * median - 1.5 * mean
EST_MEDIAN = 1       # Eq. 1
EST_MEAN = 2         # Eq. 2
EST_MODE = 3         # Eq. 4: median_factor * median - mean_factor * mean

# Per-frame flags.
FRAME_NO_VALID_MESH = 1      # no mesh node reached min_valid pixels
FRAME_EMPTY_MESH = 2         # no mesh node had any usable pixel

# Per-source flags.
SRC_APERTURE_OFF_EDGE = 1    # aperture pixel outside the frame or not finite
SRC_ANNULUS_OFF_EDGE = 2     # annulus pixel outside the frame or not finite
SRC_NO_SKY = 4               # no annulus pixel survived: sky taken as 0
SRC_INEXACT_SUM_RANGE = 8    # a pixel of the source is outside the exact range
SRC_NONPOSITIVE_FLUX = 16    # isophotal flux <= 0: unweighted centroid used
SRC_BLENDED = 32             # object split off a candidate by deblending


@dataclass
class Params:
    mesh_h: int = 64             # Sec. 2.2.2: default 64x64 regions
    mesh_w: int = 64
    filter_h: int = 3            # median filter of the mesh
    filter_w: int = 3
    clip_iters: int = 3
    clip_sigma: float = 3.0
    estimator: int = EST_SEXTRACTOR
    median_factor: float = 3.0   # Eq. 4 weights
    mean_factor: float = 2.0
    min_valid: int = 100         # Sec. 2.2.2: at least 100 pixels per region
    det_nsigma: float = 1.5
    min_area: int = 5
    connectivity: int = 8
    r_ap: float = 5.0
    r_in: float = 8.0
    r_out: float = 12.0
    sky_clip_iters: int = 3
    sky_clip_sigma: float = 3.0
    # deblending and cleaning (Sec. 2.2.5); SExtractor's usual settings
    deblend_nthresh: int = 32    # levels between threshold and peak
    deblend_mincont: float = 0.005   # flux fraction of a separate branch
    deblend_clean: bool = True
    clean_param: float = 1.0     # scale of the neighbours' modelled light
