"""CPU checks of the C-ABI library: it loads, and exports every entry point
that include/hough.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hough.h")
LIB = os.path.join(ROOT, "paper_1305_4855_amd", "libhough.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hough_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_1305_4855_amd import build
        build.build()
    return LIB


def test_header_declares_the_path():
    fns = declared_functions()
    for name in ("hough_vote", "hough_peaks", "hough_assign", "hough_prep", "hough_plan_create"):
        assert name in fns


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (hough_[a-z0-9_]+)", out))
    assert set(declared_functions()) <= exported


def test_binding_names_match_header(lib_path):
    from paper_1305_4855_amd import hough as H
    assert sorted(H.EXPORTED) == [f for f in declared_functions() if f in H.EXPORTED]
    assert set(H.EXPORTED) == set(declared_functions())


def test_library_is_gfx950_code_object(lib_path):
    data = open(lib_path, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_strerror_and_argument_errors_without_gpu(lib_path):
    lib = ctypes.CDLL(lib_path)
    lib.hough_strerror.restype = ctypes.c_char_p
    assert lib.hough_strerror(0) == b"ok"
    assert lib.hough_strerror(-1) == b"invalid argument"
    lib.hough_plan_create.restype = ctypes.c_int
    lib.hough_plan_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.hough_plan_create(None, None, None) == -1


PROBE_HEADER = os.path.join(ROOT, "include", "roofline_probe.h")
PROBE_LIB = os.path.join(ROOT, "paper_1305_4855_amd", "libroofline_probe.so")


def test_probe_library_exports_and_rejects_bad_arguments(lib_path):
    """The roofline micro-benchmark library exports what its header declares and refuses invalid
    arguments before any GPU call."""
    text = re.sub(r"/\*.*?\*/", "", open(PROBE_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(probe_[a-z0-9_]+)\s*\(", text)))
    assert names == ["probe_hbm", "probe_lds"]
    assert os.path.exists(PROBE_LIB)
    lib = ctypes.CDLL(PROBE_LIB)
    out = subprocess.run(["nm", "-D", "--defined-only", PROBE_LIB], capture_output=True, text=True).stdout
    assert set(names) <= set(re.findall(r"\bT (probe_[a-z0-9_]+)", out))
    d, f = ctypes.c_double(), ctypes.c_float()
    lib.probe_lds.restype = ctypes.c_int
    assert lib.probe_lds(0, 0, 1, 1, None, ctypes.byref(d), ctypes.byref(f)) == -1
    lib.probe_hbm.restype = ctypes.c_int
    lib.probe_hbm.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.probe_hbm(0, None, None, 17, 1, 1, ctypes.byref(d), ctypes.byref(f)) == -1
    assert b"amdgcn-amd-amdhsa--gfx950" in open(PROBE_LIB, "rb").read()
