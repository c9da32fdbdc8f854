"""The peak-probe entry points (include/probe.h) are exported by the library
and the binding declares exactly them; bad arguments are rejected before any
launch (no GPU needed)."""
import ctypes as C
import os
import re

from paper_2502_11129_amd import probe as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_probe_symbol():
    src = open(os.path.join(ROOT, "include", "probe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decl = set(re.findall(r"\b(probe_[a-z0-9_]+)\s*\(", src))
    assert decl == set(P.EXPORTED)
    lib = P.load()
    for name in decl:
        assert hasattr(lib, name), name


def test_bad_arguments_are_rejected_without_a_launch():
    lib = P.load()
    r = C.c_double()
    assert lib.probe_fp32_fma(None, 1, 1, None, C.byref(r)) == -1
    assert b"bad argument" in lib.probe_last_error()
    assert lib.probe_bf16_mfma(C.c_void_p(16), 0, 1, None, C.byref(r)) == -1
    assert lib.probe_copy(C.c_void_p(16), C.c_void_p(4096), 24, None, C.byref(r)) == -1      # not a multiple of 16
    assert lib.probe_copy(C.c_void_p(4096), C.c_void_p(4096 + 16), 64, None, C.byref(r)) == -1  # overlap
    assert b"overlap" in lib.probe_last_error()
    assert lib.probe_sincos(None, C.c_void_p(16), C.c_void_p(32), 4, None) == -1
    assert lib.probe_sincos(C.c_void_p(16), C.c_void_p(32), C.c_void_p(48), 0, None) == -1
    assert b"probe_sincos" in lib.probe_last_error()
