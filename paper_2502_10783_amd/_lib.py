"""ctypes mirror of include/ipp.h and the loader of libipp.so.

Argument marshalling only: every step of the pre-processing path runs in
the HIP kernels of libipp.so.  Loading fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# IPP_LIB: another build of the library (e.g. the host-sanitized one)
LIB_PATH = os.environ.get("IPP_LIB") or os.path.join(_HERE, "libipp.so")

IPP_OK = 0
IPP_E_INVALID_ARG = -1
IPP_E_UNSUPPORTED = -2
IPP_E_CAPACITY = -3
IPP_E_DEVICE = -4
IPP_E_WORKSPACE = -5

IPP_EST_SEXTRACTOR, IPP_EST_MEDIAN, IPP_EST_MEAN, IPP_EST_MODE = 0, 1, 2, 3
IPP_F_WRITE_RMS = 1
IPP_F_NO_GRAPH = 2
IPP_F_NO_PHOTOMETRY = 4
IPP_F_REFINE_PHOTOMETRY = 8
IPP_TUNE_MESH = 1
IPP_TUNE_TILE = 2
IPP_MAP_LINEAR, IPP_MAP_LOG, IPP_MAP_EXP, IPP_MAP_POWER = 0, 1, 2, 3
IPP_FRAME_NO_VALID_MESH = 1
IPP_FRAME_EMPTY_MESH = 2
IPP_SRC_APERTURE_OFF_EDGE = 1
IPP_SRC_ANNULUS_OFF_EDGE = 2
IPP_SRC_NO_SKY = 4
IPP_SRC_INEXACT_SUM_RANGE = 8
IPP_SRC_NONPOSITIVE_FLUX = 16
IPP_SRC_BLENDED = 32


class IppParams(C.Structure):
    _fields_ = [
        ("mesh_h", C.c_int32), ("mesh_w", C.c_int32),
        ("filter_h", C.c_int32), ("filter_w", C.c_int32),
        ("clip_iters", C.c_int32), ("estimator", C.c_int32),
        ("clip_sigma", C.c_double),
        ("median_factor", C.c_double), ("mean_factor", C.c_double),
        ("min_valid", C.c_int32), ("min_area", C.c_int32),
        ("det_nsigma", C.c_double),
        ("connectivity", C.c_int32), ("sky_clip_iters", C.c_int32),
        ("sky_clip_sigma", C.c_double),
        ("r_ap", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double),
        ("tile_h", C.c_int32), ("tile_w", C.c_int32),
        ("flags", C.c_uint32), ("reserved", C.c_int32),
    ]


class IppFrame(C.Structure):
    _fields_ = [("pix", C.c_void_p), ("mask", C.c_void_p),
                ("pitch", C.c_int64), ("h", C.c_int32), ("w", C.c_int32)]


class IppMaps(C.Structure):
    _fields_ = [("bkg", C.c_void_p), ("rms", C.c_void_p),
                ("labels", C.c_void_p)]


class IppMesh(C.Structure):
    _fields_ = [("bkg_raw", C.c_void_p), ("rms_raw", C.c_void_p),
                ("n_used", C.c_void_p), ("bkg", C.c_void_p),
                ("rms", C.c_void_p)]


class IppDeblendParams(C.Structure):
    _fields_ = [("nthresh", C.c_int32), ("clean", C.c_int32),
                ("mincont", C.c_double), ("clean_param", C.c_double)]


class IppAutoParams(C.Structure):
    _fields_ = [("kron_factor", C.c_double), ("kron_min", C.c_double),
                ("search", C.c_double)]


class IppSubtractParams(C.Structure):
    _fields_ = [("half_width", C.c_int32), ("stamp", C.c_int32),
                ("n_gauss", C.c_int32), ("spatial_order", C.c_int32),
                ("bkg_order", C.c_int32), ("order", C.c_int32 * 4),
                ("sigma", C.c_double * 4)]


SOURCE_COLUMNS = (
    ("frame", "int32"), ("label", "int32"), ("npix", "int32"),
    ("xmin", "int32"), ("xmax", "int32"), ("ymin", "int32"),
    ("ymax", "int32"), ("peak_x", "int32"), ("peak_y", "int32"),
    ("peak", "float64"), ("flux_iso", "float64"), ("x", "float64"),
    ("y", "float64"), ("flux_ap", "float64"), ("sky", "float64"),
    ("area_ap", "float64"), ("area_ann", "float64"), ("flags", "uint32"),
)


class IppSources(C.Structure):
    _fields_ = ([("capacity", C.c_int64), ("n_total", C.c_void_p),
                 ("frame_offsets", C.c_void_p)]
                + [(name, C.c_void_p) for name, _ in SOURCE_COLUMNS])


_lib = None


def lib():
    """The loaded libipp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_2502_10783_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.ipp_version.restype = i32
    L.ipp_status_string.restype = C.c_char_p
    L.ipp_status_string.argtypes = [i32]
    L.ipp_params_default.argtypes = [C.POINTER(IppParams)]
    L.ipp_params_default.restype = None
    L.ipp_params_validate.argtypes = [C.POINTER(IppParams)]
    L.ipp_params_validate.restype = i32
    L.ipp_ctx_create.argtypes = [C.POINTER(vp), i32]
    L.ipp_ctx_create.restype = i32
    L.ipp_ctx_destroy.argtypes = [vp]
    L.ipp_ctx_destroy.restype = i32
    L.ipp_ctx_reserve.argtypes = [vp, sz]
    L.ipp_ctx_reserve.restype = i32
    L.ipp_last_error.argtypes = [vp]
    L.ipp_last_error.restype = C.c_char_p
    L.ipp_ctx_profile.argtypes = [vp, i32]
    L.ipp_ctx_profile.restype = i32
    L.ipp_ctx_profile_read.argtypes = [vp, i32, C.c_char_p,
                                       C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]
    L.ipp_ctx_profile_read.restype = i32
    L.ipp_workspace_bytes.argtypes = [C.POINTER(IppFrame), i32,
                                      C.POINTER(IppParams), i64]
    L.ipp_workspace_bytes.restype = sz
    L.ipp_background.argtypes = [vp, C.POINTER(IppFrame), i32,
                                 C.POINTER(IppParams), C.POINTER(IppMaps),
                                 C.POINTER(IppMesh), vp, vp]
    L.ipp_background.restype = i32
    L.ipp_detect.argtypes = [vp, C.POINTER(IppFrame), i32,
                             C.POINTER(IppParams), C.POINTER(IppMaps),
                             C.POINTER(IppSources), vp, vp]
    L.ipp_detect.restype = i32
    L.ipp_photometry.argtypes = [vp, C.POINTER(IppFrame), i32,
                                 C.POINTER(IppMaps), C.POINTER(IppParams),
                                 C.POINTER(IppSources), vp, vp]
    L.ipp_photometry.restype = i32
    L.ipp_process_batch.argtypes = [vp, C.POINTER(IppFrame), i32,
                                    C.POINTER(IppParams), C.POINTER(IppMaps),
                                    C.POINTER(IppSources), vp, vp, vp]
    L.ipp_process_batch.restype = i32
    L.ipp_photometry_backward.argtypes = [vp, C.POINTER(IppFrame), i32,
                                          C.POINTER(IppMaps),
                                          C.POINTER(IppParams),
                                          C.POINTER(IppSources), vp, vp,
                                          C.POINTER(vp), vp, vp]
    L.ipp_photometry_backward.restype = i32
    L.ipp_refine_workspace_bytes.argtypes = [C.POINTER(IppFrame), i32, i64]
    L.ipp_refine_workspace_bytes.restype = sz
    L.ipp_refine_centroids.argtypes = [vp, C.POINTER(IppFrame), i32,
                                       C.POINTER(IppMaps),
                                       C.POINTER(IppParams),
                                       C.POINTER(IppSources), C.c_double,
                                       C.c_double, i32, vp, vp, vp]
    L.ipp_refine_centroids.restype = i32
    L.ipp_asinh.argtypes = [vp, vp, vp, i64, C.c_double, C.c_double, vp]
    L.ipp_asinh.restype = i32
    L.ipp_asinh_backward.argtypes = [vp, vp, vp, vp, vp, i64, C.c_double,
                                     C.c_double, vp]
    L.ipp_asinh_backward.restype = i32
    L.ipp_asinh_dev.argtypes = [vp, vp, vp, i64, vp, vp]
    L.ipp_asinh_dev.restype = i32
    L.ipp_asinh_backward_dev.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
    L.ipp_asinh_backward_dev.restype = i32
    L.ipp_asinh_backward_noalloc.argtypes = [vp, vp, vp, vp, vp, i64,
                                             C.c_double, C.c_double, vp]
    L.ipp_asinh_backward_noalloc.restype = i32
    L.ipp_autotune.argtypes = [vp, C.POINTER(IppFrame), i32,
                               C.POINTER(IppParams), C.c_uint32, C.c_char_p,
                               C.POINTER(C.c_double), vp]
    L.ipp_autotune.restype = i32
    L.ipp_deblend_params_default.argtypes = [C.POINTER(IppDeblendParams)]
    L.ipp_deblend_params_default.restype = None
    L.ipp_deblend_workspace_bytes.argtypes = [C.POINTER(IppFrame), i32, i64,
                                              i64]
    L.ipp_deblend_workspace_bytes.restype = sz
    L.ipp_deblend.argtypes = [vp, C.POINTER(IppFrame), i32,
                              C.POINTER(IppParams),
                              C.POINTER(IppDeblendParams), C.POINTER(IppMaps),
                              C.POINTER(IppSources), C.POINTER(vp),
                              C.POINTER(IppSources), vp, vp, vp]
    L.ipp_deblend.restype = i32
    L.ipp_auto_params_default.argtypes = [C.POINTER(IppAutoParams)]
    L.ipp_auto_params_default.restype = None
    L.ipp_photometry_auto.argtypes = [vp, C.POINTER(IppFrame), i32,
                                      C.POINTER(IppMaps),
                                      C.POINTER(IppSources), vp,
                                      C.POINTER(IppAutoParams), vp, vp, vp,
                                      vp, vp]
    L.ipp_photometry_auto.restype = i32
    L.ipp_subtract_params_default.argtypes = [
        C.POINTER(IppSubtractParams)]
    L.ipp_subtract_params_default.restype = None
    L.ipp_subtract_coef_count.argtypes = [C.POINTER(IppSubtractParams)]
    L.ipp_subtract_coef_count.restype = i64
    L.ipp_subtract.argtypes = [vp, C.POINTER(IppFrame), C.POINTER(IppFrame),
                               i32, C.POINTER(IppSubtractParams), vp,
                               C.POINTER(vp), vp]
    L.ipp_subtract.restype = i32
    L.ipp_source_moments.argtypes = [vp, C.POINTER(IppFrame), i32,
                                     C.POINTER(IppMaps), C.POINTER(IppSources),
                                     vp, vp]
    L.ipp_source_moments.restype = i32
    L.ipp_gray_workspace_bytes.argtypes = [i32, i32]
    L.ipp_gray_workspace_bytes.restype = sz
    L.ipp_zscale.argtypes = [vp, C.POINTER(IppFrame), i32, i32, C.c_double,
                             vp, vp, vp]
    L.ipp_zscale.restype = i32
    L.ipp_gray_map.argtypes = [vp, C.POINTER(IppFrame), i32, i32, C.c_double,
                               vp, C.POINTER(vp), vp]
    L.ipp_gray_map.restype = i32
    L.ipp_equalize.argtypes = [vp, C.POINTER(IppFrame), i32, i32,
                               C.POINTER(vp), vp, vp]
    L.ipp_equalize.restype = i32
    _lib = L
    return L


def header_functions():
    """Names of the functions include/ipp.h declares."""
    import re
    path = os.path.join(os.path.dirname(_HERE), "include", "ipp.h")
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ipp_[a-z_0-9]+)\s*\(", text)))
