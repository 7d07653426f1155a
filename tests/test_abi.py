"""CPU checks of the C ABI: the built library loads and exports every entry point
that include/mfg.h declares, and the binding declares exactly those. No
compute call is made (there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfg.h")
LIB = os.path.join(ROOT, "paper_2507_01958_amd", "libmfg.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfg_[a-z0-9_A-Z]+)\s*\(", text)))


def test_header_declares_the_api():
    names = header_functions()
    for required in ["mfg_plan", "mfg_prox", "mfg_apply_AAt", "mfg_precond", "mfg_pcg",
                     "mfg_cp_solve", "mfg_destroy", "mfg_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfg.so not built")
def test_library_exports_every_header_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_matches_header():
    from paper_2507_01958_amd import mfg
    assert sorted(mfg.SIGNATURES) == header_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfg.so not built")
def test_version_and_error_without_gpu():
    from paper_2507_01958_amd import mfg
    lib = mfg.load()
    assert b"gfx950" in lib.mfg_version()
    # invalid arguments are rejected on the host before any device work
    h = ctypes.c_void_p()
    pb = mfg.make_problem(3, 8, 8, 4, "periodic", 0.1, 5e-4)
    rc = lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h))
    assert rc == 1 and b"d must be" in lib.mfg_last_error()
    pb = mfg.make_problem(2, 10, 8, 4, "periodic", 0.1, 5e-4)
    assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 2
    for qp in (1.0, 1.1, 8.0):   # q' outside the supported range [1.2, 6]
        pb = mfg.make_problem(2, 8, 8, 4, "periodic", 0.1, 5e-4, qprime=qp)
        assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 2
    # a boundary type per axis needs d = 2; unknown codes are rejected
    pb = mfg.make_problem(1, 8, 1, 4, ("periodic", "neumann"), 0.1, 5e-4)
    assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 1
    pb = mfg.make_problem(2, 8, 8, 4, 4, 0.1, 5e-4)
    assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 1
    # cells of an n-vector are indexed with 32-bit arithmetic: n < 2^31
    pb = mfg.make_problem(2, 1024, 1024, 2048, "periodic", 0.1, 5e-4)
    assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 2
    assert b"grid too large" in lib.mfg_last_error()
    pb = mfg.make_problem(2, 8, 8, 4, "periodic", -1.0, 5e-4)
    assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 1
    pb = mfg.make_problem(2, 8, 8, 4, "periodic", 0.1, 5e-4, l=3)
    assert lib.mfg_plan(ctypes.byref(pb), None, None, None, ctypes.byref(h)) == 1
    assert lib.mfg_prox(None, None, 1.0, None) == 1
    assert lib.mfg_destroy(None) == 0
