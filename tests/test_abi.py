"""The C-ABI library loads and exports every symbol its header declares (no GPU calls)."""
import ctypes
import os

import pytest

from paper_1703_05638_amd import lrpost as lp


def test_header_declares_the_boundary():
    names = lp.header_symbols()
    for must in ["lrpost_create", "lrpost_destroy", "lrpost_hess_apply", "lrpost_eigensolve",
                 "lrpost_post_variance", "lrpost_sample", "lrpost_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lp.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(lp.LIB_PATH)
    missing = [n for n in lp.header_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_path_without_gpu_work():
    if not os.path.exists(lp.LIB_PATH):
        pytest.skip("library not built")
    lib = lp.load()
    # invalid descriptions are rejected on the host before any device work
    d = lp.Desc()
    d.N, d.nt, d.T, d.alpha, d.sigma = 30, 10, 1.0, 1e-2, 1e-2
    d.trunc_tol, d.rank_cap = 1e-6, 8
    h = ctypes.c_void_p()
    rc = lib.lrpost_create(ctypes.byref(d), ctypes.byref(h))
    assert rc == -1
    assert b"power of two" in lib.lrpost_last_error()


def test_rejections_before_device_work():
    """mg_levels other than 0, null handles and negative limits are refused
    with LRPOST_EINVAL before anything touches the device."""
    if not os.path.exists(lp.LIB_PATH):
        pytest.skip("library not built")
    lib = lp.load()
    d = lp.Desc()
    d.N, d.nt, d.T, d.alpha, d.sigma = 32, 10, 1.0, 1e-2, 1e-2
    d.box[0], d.box[1], d.box[2], d.box[3] = 0.25, 0.75, 0.25, 0.75
    d.trunc_tol, d.rank_cap, d.mg_levels = 1e-6, 8, 4
    h = ctypes.c_void_p()
    assert lib.lrpost_create(ctypes.byref(d), ctypes.byref(h)) == -1
    assert b"mg_levels" in lib.lrpost_last_error()
    assert lib.lrpost_set_eig_limits(None, 8, 0.0) == -1
    assert lib.lrpost_set_st_check(None, 1, 0.0) == -1
    res = (ctypes.c_double * 1)()
    assert lib.lrpost_eig_residuals(None, None, res) == -1
    rates = (ctypes.c_double * 2)()
    assert lib.lrpost_measure_fp64_rates(0, rates) == -1
    assert lib.lrpost_measure_fp64_rates(100001, rates) == -1
    assert lib.lrpost_measure_fp64_rates(10, None) == -1
