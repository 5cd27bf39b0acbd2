"""The C ABI library without a GPU: it loads, exports every function that
include/ipp.h declares, and validates arguments on the host."""
import ctypes as C

import pytest

from paper_2502_10783_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_exports_every_declared_function(lib):
    names = L.header_functions()
    assert "ipp_process_batch" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_status_strings(lib):
    assert lib.ipp_version() == 1
    assert lib.ipp_status_string(L.IPP_E_WORKSPACE) == b"workspace too small"
    assert lib.ipp_status_string(123) == b"unknown status"


def _defaults(lib):
    p = L.IppParams()
    lib.ipp_params_default(C.byref(p))
    return p


def test_defaults_are_the_papers(lib):
    p = _defaults(lib)
    assert (p.mesh_h, p.mesh_w, p.filter_h, p.filter_w) == (64, 64, 3, 3)
    assert (p.clip_iters, p.clip_sigma, p.min_valid) == (3, 3.0, 100)
    assert (p.det_nsigma, p.min_area, p.connectivity) == (1.5, 5, 8)
    assert (p.r_ap, p.r_in, p.r_out) == (5.0, 8.0, 12.0)
    assert lib.ipp_params_validate(C.byref(p)) == L.IPP_OK


@pytest.mark.parametrize("field,value", [
    ("mesh_h", 8), ("mesh_w", 256), ("filter_h", 2), ("filter_w", 9),
    ("clip_iters", -1), ("clip_sigma", 0.0), ("estimator", 7),
    ("min_valid", 0), ("min_area", 0), ("connectivity", 6),
    ("sky_clip_sigma", -1.0), ("r_ap", 0.0), ("r_in", 12.0),
    ("r_out", 40.0), ("tile_h", 48), ("det_nsigma", float("nan")),
])
def test_invalid_params_rejected(lib, field, value):
    p = _defaults(lib)
    setattr(p, field, value)
    assert lib.ipp_params_validate(C.byref(p)) == L.IPP_E_INVALID_ARG
    assert lib.ipp_params_validate(None) == L.IPP_E_INVALID_ARG


def _frames(shapes):
    arr = (L.IppFrame * len(shapes))()
    for i, (h, w) in enumerate(shapes):
        arr[i].pix = 0x1000 * (i + 1)          # never dereferenced
        arr[i].pitch = w
        arr[i].h, arr[i].w = h, w
    return arr


def test_workspace_bytes_host_only(lib):
    p = _defaults(lib)
    f = _frames([(1024, 1024), (100, 333)])
    n0 = lib.ipp_workspace_bytes(f, 2, C.byref(p), 0)
    n1 = lib.ipp_workspace_bytes(f, 2, C.byref(p), 1 << 20)
    assert n0 > 2 * (1024 * 1024 + 100 * 333) and n1 > n0
    f[1].pitch = 10                              # pitch < w
    assert lib.ipp_workspace_bytes(f, 2, C.byref(p), 0) == 0
    f = _frames([(0, 5)])
    assert lib.ipp_workspace_bytes(f, 1, C.byref(p), 0) == 0
    assert lib.ipp_workspace_bytes(None, 1, C.byref(p), 0) == 0


def test_null_context_rejected(lib):
    p = _defaults(lib)
    f = _frames([(64, 64)])
    maps = (L.IppMaps * 1)()
    src = L.IppSources()
    assert lib.ipp_background(None, f, 1, C.byref(p), maps, None, None,
                              None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_detect(None, f, 1, C.byref(p), maps, C.byref(src), None,
                          None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_photometry(None, f, 1, maps, C.byref(p), C.byref(src),
                              None, None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_process_batch(None, f, 1, C.byref(p), maps, C.byref(src),
                                 None, None, None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_ctx_destroy(None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_ctx_create(None, 0) == L.IPP_E_INVALID_ARG


def test_gray_workspace_and_argument_checks(lib):
    assert lib.ipp_gray_workspace_bytes(0, 0) == 0
    assert lib.ipp_gray_workspace_bytes(2, 1) == 0
    assert lib.ipp_gray_workspace_bytes(2, 4097) == 0
    n0 = lib.ipp_gray_workspace_bytes(16, 0)
    n1 = lib.ipp_gray_workspace_bytes(16, 4096)
    assert n0 > 0 and n1 >= n0 + 16 * 4096 * (4 + 8)
    f = _frames([(64, 64)])
    z = C.c_void_p(1)
    assert lib.ipp_zscale(None, f, 1, 1000, 0.25, z, None,
                          None) == L.IPP_E_INVALID_ARG
    outs = (C.c_void_p * 1)(1)
    assert lib.ipp_gray_map(None, f, 1, L.IPP_MAP_LOG, 1000.0, z, outs,
                            None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_equalize(None, f, 1, 4096, outs, None,
                            None) == L.IPP_E_INVALID_ARG


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library the binding refuses to run (no fallback)."""
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libipp.so")
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()


def test_deblend_kron_refine_host_checks(lib):
    d = L.IppDeblendParams()
    lib.ipp_deblend_params_default(C.byref(d))
    assert (d.nthresh, d.clean, d.mincont, d.clean_param) == \
        (32, 1, 0.005, 1.0)
    a = L.IppAutoParams()
    lib.ipp_auto_params_default(C.byref(a))
    assert (a.kron_factor, a.kron_min, a.search) == (2.5, 3.5, 6.0)
    f = _frames([(128, 96), (64, 64)])
    w0 = lib.ipp_deblend_workspace_bytes(f, 2, 1000, 0)
    w1 = lib.ipp_deblend_workspace_bytes(f, 2, 1000, 1 << 20)
    assert w0 > 4 * 8 * 1000 and w1 >= w0 + (1 << 20)
    assert lib.ipp_deblend_workspace_bytes(f, 2, -1, 0) == 0
    assert lib.ipp_deblend_workspace_bytes(None, 2, 10, 0) == 0
    r0 = lib.ipp_refine_workspace_bytes(f, 2, 1000)
    assert r0 > 0 and lib.ipp_refine_workspace_bytes(f, 2, 10) == r0
    assert lib.ipp_refine_workspace_bytes(f, 2, -5) == 0
    p = _defaults(lib)
    maps = (L.IppMaps * 2)()
    src = L.IppSources()
    outs = (C.c_void_p * 2)(1, 2)
    assert lib.ipp_deblend(None, f, 2, C.byref(p), C.byref(d), maps,
                           C.byref(src), outs, C.byref(src), None, None,
                           None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_photometry_auto(None, f, 2, maps, C.byref(src), None,
                                   None, None, None, None, None,
                                   None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_refine_centroids(None, f, 2, maps, C.byref(p),
                                    C.byref(src), 2.0, 3.0, 10, None, None,
                                    None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_asinh_dev(None, None, None, 0, None,
                             None) == L.IPP_E_INVALID_ARG
    assert lib.ipp_asinh_backward_noalloc(None, None, None, None, None, 0,
                                          1.0, 1.0,
                                          None) == L.IPP_E_INVALID_ARG


def test_binding_constants_match_the_header():
    """Every IPP_ macro of include/ipp.h with a plain integer value that the
    binding also names has the same value there (flags, per-source and
    per-frame bits)."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include",
                            "ipp.h")).read()
    seen = 0
    for name, val in re.findall(r"#define\s+(IPP_\w+)\s+(\d+)u?\b", hdr):
        if hasattr(L, name):
            assert getattr(L, name) == int(val), name
            seen += 1
    assert L.IPP_F_NO_PHOTOMETRY == 4 and L.IPP_F_REFINE_PHOTOMETRY == 8
    assert seen >= 4
