"""The C-ABI library loads and exports every function include/nhswe.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nhswe.h")
LIB = os.path.join(ROOT, "paper_1706_04551_amd", "_lib", "libnhswe.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(nh_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("nh_create", "nh_set_bathymetry", "nh_set_state", "nh_step",
                 "nh_run", "nh_read_state", "nh_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.nh_version.restype = ctypes.c_char_p
    assert lib.nh_version().startswith(b"nhswe")


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_invalid_arguments_are_rejected_without_a_device():
    from paper_1706_04551_amd import binding as B
    L = B.lib()
    out = ctypes.c_void_p()
    g = B.NhGrid(1, 1, 1.0, 1.0)           # nx < 2
    p = B.NhParams(9.81, 0.9, 1e-5, 1e-10, 0, 1, 0, 0.15, 0.5, 10, 1, 1e-10,
                   None, 0, 0, 0.0)
    assert L.nh_create(ctypes.byref(g), ctypes.byref(p), None,
                       ctypes.byref(out)) == -1
    assert b"nx" in L.nh_last_error()
    g = B.NhGrid(10, 10, 1.0, 1.0)
    p.cfl = 1.5
    assert L.nh_create(ctypes.byref(g), ctypes.byref(p), None,
                       ctypes.byref(out)) == -1
    p.cfl = 0.9
    p.check_every = 3
    om = (ctypes.c_double * 2)(1.0, 2.0)
    p.omega_schedule = ctypes.cast(om, ctypes.POINTER(ctypes.c_double))
    p.n_omega = 2
    assert L.nh_create(ctypes.byref(g), ctypes.byref(p), None,
                       ctypes.byref(out)) == -1
    assert b"multiple" in L.nh_last_error()
    p.check_every, p.n_omega = 1, 0
    p.omega_schedule = None
    p.manning = -0.01                      # friction coefficient
    assert L.nh_create(ctypes.byref(g), ctypes.byref(p), None,
                       ctypes.byref(out)) == -1
    assert b"manning" in L.nh_last_error()
    p.manning, p.open_sides = 0.0, 16      # outflow mask of 4 bits
    assert L.nh_create(ctypes.byref(g), ctypes.byref(p), None,
                       ctypes.byref(out)) == -1
    assert b"open_sides" in L.nh_last_error()
    assert L.nh_step(None, None) == -1
    assert L.nh_bind_device_buffers(None, None) == -1
    assert L.nh_set_relaxation(None, None, None, None, None, None,
                               None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_ensemble_arguments_are_checked_without_a_device():
    from paper_1706_04551_amd import binding as B
    L = B.lib()
    out = ctypes.c_void_p()

    def params(prec=0):
        return B.NhParams(9.81, 0.7, 1e-5, 1e-10, prec, 1, 0, 0.15, 0.5, 100,
                          1, 1e-10, None, 0, 0, 0.0)
    G = (B.NhGrid * 2)(B.NhGrid(10, 10, 1.0, 1.0), B.NhGrid(12, 12, 1.0, 1.0))
    P = (B.NhParams * 2)(params(0), params(1))
    assert L.nh_ensemble_create(2, G, P, None, ctypes.byref(out)) == -1
    assert b"share" in L.nh_last_error()
    P = (B.NhParams * 2)(params(0), params(0))
    G1 = (B.NhGrid * 2)(B.NhGrid(10, 10, 1.0, 1.0), B.NhGrid(12, 1, 1.0, 1.0))
    assert L.nh_ensemble_create(2, G1, P, None, ctypes.byref(out)) == -1
    assert b"2D" in L.nh_last_error()
    assert L.nh_ensemble_create(0, G, P, None, ctypes.byref(out)) == -1
    assert L.nh_ensemble_run(None, 1) == -1
    assert L.nh_ensemble_set_tile(None, 0, 24, 24) == -1
