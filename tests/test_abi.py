"""The C-ABI library loads and exports every symbol include/gd.h declares;
host-side validation rejects bad input before any device work (CPU only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gd.h")
LIB = os.path.join(ROOT, "paper_1901_06363_amd", "libgd.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gd_status|const char\*)\s+(gd_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("gd_create_pocket", "gd_dock_batch", "gd_score_poses", "gd_refine", "gd_last_error",
                 "gd_surrogate_fwd", "gd_surrogate_bwd", "gd_destroy_pocket"):
        assert need in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first"
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB]).decode()
    exported = set(re.findall(r" T (gd_\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        getattr(lib, n)


def test_binding_signatures_cover_the_header():
    from paper_1901_06363_amd import _abi
    assert sorted(n for n, _, _ in _abi.SIGNATURES) == declared_functions()


def test_pocket_validation_errors_without_device_work():
    from paper_1901_06363_amd import _abi
    lib = _abi.load()
    pts = np.zeros((4, 3), np.float32)
    h = ctypes.c_void_p()

    def mk(**kw):
        d = dict(xyz=pts.ctypes.data_as(ctypes.c_void_p), n_points=4, grid_h=0.5, pad=12.0, blur_sigma=0.0,
                 blur_h=0.375, blur_cutoff_sigmas=4.0, blur_pad=8.0)
        d.update(kw)
        return _abi.PocketDesc(**d)

    assert lib.gd_create_pocket(None, None, ctypes.byref(h)) == 1
    assert lib.gd_last_error().decode().startswith("gd_create_pocket")
    assert lib.gd_create_pocket(ctypes.byref(mk(grid_h=0.3)), None, ctypes.byref(h)) == 1
    assert "power of two" in lib.gd_last_error().decode()
    assert lib.gd_create_pocket(ctypes.byref(mk(n_points=0)), None, ctypes.byref(h)) == 1
    assert lib.gd_create_pocket(ctypes.byref(mk(pad=-1.0)), None, ctypes.byref(h)) == 1
    big = np.array([[0, 0, 0], [400, 0, 0]], np.float32)
    d = mk(xyz=big.ctypes.data_as(ctypes.c_void_p), n_points=2)
    assert lib.gd_create_pocket(ctypes.byref(d), None, ctypes.byref(h)) == 7  # > 512 cells per axis
    assert not h.value
