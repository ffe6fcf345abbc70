"""Host-side checks of the C ABI: the library loads, exports every declared entry point,
validates parameters and reproduces the oracle's level tables bit for bit.  No GPU."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from oracle import ridge_hough as O
from paper_1310_1371_amd import native as N
from paper_1310_1371_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(N.LIB_PATH):
        from paper_1310_1371_amd import build
        build.build(verbose=False)
    return N.lib()


def _declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w\s\*]*?\b(rd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported_and_bound():
    lib = _ensure_built()
    names = _declared()
    assert "rd_detect" in names and "rd_create" in names
    for name in names:
        assert hasattr(lib, name), name
        assert name in N.SIGNATURES, name


def test_status_strings():
    _ensure_built()
    assert N.status_string(N.RD_OK) == "ok"
    assert "invalid" in N.status_string(N.RD_E_INVALID)


def _p(**kw):
    return N.make_params(dict(O.DEFAULTS, **kw))


@pytest.mark.parametrize("kw,ok", [
    ({}, True),
    (dict(sigma_smooth=0.0), False), (dict(sigma_smooth=4.5), False),
    (dict(k_threshold=0.1), False), (dict(k_threshold=float("nan")), False),
    (dict(r_min=0), False), (dict(r_min=10, r_max=9), False), (dict(r_max=127), False),
    (dict(r_max=126), True), (dict(vote_threshold=-1), False),
    (dict(peak_fraction=-0.1), False), (dict(sig_slope=-0.01), False), (dict(sig_icpt=0.0), False),
    (dict(sig_slope=0.2, r_max=126), False),
    (dict(annulus_halfwidth=-1), False), (dict(min_fit_points=2), False),
    (dict(r_step=0), True), (dict(r_step=3), True), (dict(r_step=-1), False), (dict(r_step=17), False),
    (dict(r_min=4, r_step=4), False), (dict(r_min=5, r_step=4), True), (dict(r_min=1), False),
    (dict(r_min=2), True),
    (dict(r_min=100, r_max=124, r_step=3), True), (dict(r_min=100, r_max=124, r_step=4), False),
    (dict(curvature_fp32=1), True), (dict(curvature_fp32=2), False), (dict(curvature_fp32=-1), False),
])
def test_validate_params(kw, ok):
    lib = _ensure_built()
    st = lib.rd_validate_params(ctypes.byref(_p(**kw)))
    assert (st == N.RD_OK) == ok


@pytest.mark.parametrize("params", [synth.PARAMS_C1, synth.PARAMS_C2, synth.PARAMS_C5,
                                    dict(O.DEFAULTS, sig_slope=0.07, sig_icpt=0.4, peak_fraction=0.33),
                                    dict(synth.PARAMS_C2, r_step=3), dict(synth.PARAMS_C5, r_step=2)])
def test_level_tables_match_oracle(params):
    lib = _ensure_built()
    p = dict(O.DEFAULTS, **params)
    L = N.n_levels(p)
    k = np.zeros(L, np.int32)
    w = np.zeros(L * 25, np.uint32)
    t = np.zeros(L, np.uint64)
    st = lib.rd_level_tables(ctypes.byref(N.make_params(p)), L, k.ctypes.data, w.ctypes.data, t.ctypes.data)
    assert st == N.RD_OK
    radii = O.level_radii(p)
    assert len(radii) == L
    for i in range(L):
        r = int(radii[i])
        assert k[i] == O.level_radius(r, p)
        wf = O.weight_factors(r, p)
        np.testing.assert_array_equal(w[i * 25:i * 25 + len(wf)], wf)
        assert not w[i * 25 + len(wf):(i + 1) * 25].any()
        assert int(t[i]) == O.score_threshold(r, p)
    assert lib.rd_level_tables(ctypes.byref(N.make_params(p)), L - 1, None, None, None) == N.RD_E_TRUNCATED


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    lib = _ensure_built()
    info = N.RdCreateInfo(0, 256, 256, 1024, 1, 0, None)
    h = ctypes.c_void_p()
    assert lib.rd_create(ctypes.byref(info), ctypes.byref(h)) == N.RD_E_DEVICE
    assert not h.value
    bad = N.RdCreateInfo(0, 16, 256, 1024, 1, 0, None)
    assert lib.rd_create(ctypes.byref(bad), ctypes.byref(h)) == N.RD_E_INVALID
    lib.rd_destroy(None)


@pytest.mark.parametrize("gate,memory,c2,max_tracks,model", [
    (0.0, 1, 72.0, 100, 0), (-1.0, 1, 72.0, 100, 0), (float("nan"), 1, 72.0, 100, 0), (5.0, -1, 72.0, 100, 0),
    (5.0, 1, 0.0, 100, 0), (5.0, 1, float("nan"), 100, 0), (5.0, 1, 72.0, 0, 0),
    (5.0, 1, -72.0, 100, 0), (5.0, 1, float("inf"), 100, 0), (5.0, 1, 72.0, 100, 2), (5.0, 1, 72.0, 100, -1)])
def test_linker_parameters_are_validated_before_device_work(gate, memory, c2, max_tracks, model):
    lib = _ensure_built()
    h = ctypes.c_void_p()
    p = N.RdLinkParams(gate, memory, 8.0, 0.0, c2, model)
    assert lib.rd_linker_create(ctypes.byref(p), max_tracks, 4, None, ctypes.byref(h)) == N.RD_E_INVALID
    offs = (ctypes.c_int32 * 2)(0, 0)
    assert lib.rd_link(None, None, offs, 1, None, None) == N.RD_E_INVALID
    assert lib.rd_linker_reset(None) == N.RD_E_INVALID
