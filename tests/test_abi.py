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
