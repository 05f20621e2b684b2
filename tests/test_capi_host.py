"""Host-side checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import math
import os
import re

import pytest

from paper_1609_04661_amd import api, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "dgampct.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:dg_status|size_t|int64_t|int32_t|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_header_symbols():
    L = api.load()
    names = header_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(api.EXPORTS) == set(names)


def test_plan_create_rejects_bad_geometry():
    L = api.load()
    bad = [
        dict(synth.c1_geometry(), n=4),
        dict(synth.c1_geometry(), n_views=0),
        dict(synth.c1_geometry(), pixel_mm=0.0),
        dict(synth.c1_geometry(), bin_mm=-1.0),
        dict(synth.c1_geometry(), kind=7),
        dict(synth.c5_geometry(), dso_mm=100.0),
        dict(synth.c1_geometry(), span_rad=float("nan")),
        # parallel bins so narrow that bin coordinates over the image reach 2^16
        dict(synth.c2_geometry(), bin_mm=0.01, n_bins=64),
    ]
    for g in bad:
        c = api.Geom(**{k: g[k] for k, _ in api.Geom._fields_})
        h = ctypes.c_void_p()
        assert L.dg_plan_create(ctypes.byref(c), ctypes.byref(h)) == -1
        assert L.dg_last_error()
    assert b"2^16" in L.dg_last_error()
    assert L.dg_plan_create(None, None) == -1


def test_channel_rejects_bad_arguments():
    L = api.load()
    w = ctypes.c_void_p(1)
    assert L.gamp_poisson_out(0, w, w, w, 1e4, 0, w, w, w, None) == -1
    assert L.gamp_poisson_out(10, w, w, w, -1.0, 0, w, w, w, None) == -1
    assert L.gamp_poisson_out(10, w, w, w, 1e4, 9, w, w, w, None) == -1
    assert L.gamp_poisson_out(10, None, w, w, 1e4, 0, w, w, w, None) == -1
    assert b"mode" in L.dg_last_error() or b"null" in L.dg_last_error()


def test_workspace_query_null_plan():
    L = api.load()
    assert L.dg_workspace_bytes(None, 0) == 0
    assert L.dg_channel_workspace_bytes(1000) > 0


def test_tv_workspace_size():
    """The proximal-TV dual state: the perturbed input plus p and u, ping and
    pong, two components, two images: 17 planes of 256-byte-aligned floats."""
    L = api.load()
    assert L.dg_tv_workspace_bytes(0) == 0
    assert L.dg_tv_workspace_bytes(512 * 512) == 17 * 512 * 512 * 4
    assert L.dg_tv_workspace_bytes(10) == 17 * 256


def test_tvw_workspace_size():
    """The metric proximal TV's state: the perturbed input, x, xbar and two
    ping-pong copies of the two dual components per image (13 planes), and
    two half spectra of (I/2+1) x I complex floats per image (F v and F r),
    each region 256-byte aligned."""
    L = api.load()
    assert L.dg_tvw_workspace_bytes(0) == 0
    assert L.dg_tvw_workspace_bytes(512) == 13 * 512 * 512 * 4 + 4 * 257 * 512 * 8
    # side 12: 144 floats -> 768 bytes per plane; 7 x 12 complex -> 768 bytes per spectrum
    assert L.dg_tvw_workspace_bytes(12) == 13 * 768 + 4 * 768


def test_product_path_has_no_cpu_fallback():
    # the binding must not import the oracle and must refuse non-CUDA tensors
    import torch
    src = open(os.path.join(ROOT, "paper_1609_04661_amd", "api.py")).read()
    assert "oracle" not in src.replace("not compute", "")
    with pytest.raises(api.DgError):
        api._ptr(torch.zeros(4), torch.float32)


def test_batch_entry_points_reject_bad_arguments():
    """Argument checks run before any device call."""
    L = api.load()
    g = api.Geom(**{k: synth.c1_geometry()[k] for k, _ in api.Geom._fields_})
    h = ctypes.c_void_p()
    assert L.dg_batch_create(ctypes.byref(g), 0, ctypes.byref(h)) == -1
    assert L.dg_batch_create(None, 1, ctypes.byref(h)) == -1
    a = (ctypes.c_double * 1)(1.0)
    assert L.dg_batch_bind(None, None, a, a, None, None, None, None, 1, None, 1e-3, None) == -1
    assert L.dg_batch_state_init(None, 1.0, None) == -1
    assert L.dgamp_batch_iterate(None, 1, 0, 0, 1.0, 1.0, 1, 0, 0, None) == -1
    assert L.dg_batch_autotune(None, 1, None) == -1
    assert L.dg_batch_workspace_bytes(None) == 0
    assert L.dg_batch_projector_variant(None) == -1
    assert L.dg_plan_projector_variant(None) == -1
    assert L.dg_plan_autotune(None, None, None, None, 1, None) == -1
    assert L.dg_last_error()


def test_psnr_rejects_bad_arguments():
    L = api.load()
    assert L.dg_psnr_workspace_bytes() >= 8
    assert L.dg_psnr(0, None, None, None, None, None) == -1
    assert L.dg_psnr(10, None, None, None, None, None) == -1


def test_check_status_and_noalloc_reject_null_arguments():
    L = api.load()
    assert L.dg_check_status(None, 1, None, None, None) == -1
    assert L.dg_check_status(ctypes.c_void_p(8), 0, None, None, None) == -1
    assert L.dgamp_iterate_noalloc(None, None, None, None, None, None, None) == -1
    assert L.dg_noalloc_scratch_bytes() == 48 << 20
