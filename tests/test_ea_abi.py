"""Evolutionary-loop C ABI (host only, no device work): every entry point
declared in include/ea.h is exported, and invalid arguments are rejected
before anything is launched."""
import os
import re

from paper_2502_11129_amd import ea as EA

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_ea_symbol():
    src = open(os.path.join(ROOT, "include", "ea.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decl = set(re.findall(r"\b(ea_[a-z_]+)\s*\(", src))
    assert decl == set(EA.EXPORTED)
    lib = EA.load()
    for name in decl:
        assert hasattr(lib, name), name


def test_invalid_arguments_are_rejected_without_launching():
    lib = EA.load()
    n = [None] * 5
    assert lib.ea_vary(0, *n, None, 10, 1, 0, *n, None) == -1          # mu < 1
    assert b"mu" in lib.ea_last_error()
    assert lib.ea_vary(4, *n, None, -1, 1, 0, *n, None) == -1          # n_off < 0
    assert lib.ea_vary(4, *n, None, 10, 1, 0, *n, None) == -1          # NULL arrays
    assert lib.ea_vary(4, *n, None, 0, 1, 0, *n, None) == 0            # nothing to do
    assert lib.ea_tune_perturb(-1, None, None, 1, 0, 0, None, None) == -1
    assert lib.ea_tune_perturb(3, None, None, 1, 0, 0, None, None) == -1
    assert lib.ea_tune_accept(3, None, None, None, None, None) == -1
    assert lib.ea_gather(2, None, 1, *n, None, 0, *n, None, *n, None, None) == -1
    assert lib.ea_gather(0, None, 1, *n, None, 0, *n, None, *n, None, None) == 0
