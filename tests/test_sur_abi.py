"""Surrogate C ABI (host only, no device work): every entry point declared in
include/sur.h is exported, and sur_create validates its configuration."""
import ctypes as C
import os
import re

import pytest

from paper_2502_11129_amd import surrogate as SU

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_surrogate_symbol():
    src = open(os.path.join(ROOT, "include", "sur.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decl = set(re.findall(r"\b(sur_[a-z_]+)\s*\(", src))
    assert decl == set(SU.EXPORTED)
    lib = SU.load()
    for name in decl:
        assert hasattr(lib, name), name


def _create(**kw):
    lib = SU.load()
    cfg = SU.sur_config(kw.get("max_batch", 4096), 0, kw.get("lr", 1e-3), kw.get("beta1", 0.9),
                        kw.get("beta2", 0.999), kw.get("eps", 1e-8))
    h = C.c_void_p()
    rc = lib.sur_create(C.byref(cfg), C.byref(h))
    return lib, rc, h


def test_create_validates_and_reports_workspace():
    lib, rc, h = _create()
    assert rc == 0
    b = C.c_size_t()
    assert lib.sur_workspace_bytes(h, C.byref(b)) == 0
    # parameters, moments, gradients and copies, plus activations of 65536 rows
    assert b.value > 4 * 4 * SU.SUR_N_PARAMS + 65536 * 256 * 2 * 5
    # calls before sur_bind are refused
    assert lib.sur_predict(h, 1, None, 1, None, None, None) == -4
    assert b"sur_bind" in lib.sur_last_error(h)
    lib.sur_destroy(h)
    for bad in (dict(max_batch=0), dict(max_batch=70000), dict(lr=0.0), dict(beta1=1.0), dict(beta2=-0.1),
                dict(eps=0.0)):
        lib, rc, h = _create(**bad)
        assert rc == -1, bad
        assert h.value is None
        assert len(lib.sur_last_error(None)) > 0


def test_noalloc_topk_refuses_sizes_beyond_its_scratch():
    """sur_topk_noalloc rejects n above its static scratch, and k outside
    [0, n], with a message and before any device call."""
    import ctypes as C
    from paper_2502_11129_amd import surrogate as SU
    lib = SU.load()
    err = C.create_string_buffer(256)
    rc = lib.sur_topk_noalloc(SU.SUR_TOPK_NOALLOC_MAX + 1, None, 1, None, None, err, 256)
    assert rc == -1 and b"SUR_TOPK_NOALLOC_MAX" in err.value
    rc = lib.sur_topk_noalloc(10, None, 11, None, None, err, 256)
    assert rc == -1 and b"k <= n" in err.value
    assert lib.sur_topk_noalloc(10, None, 0, None, None, None, 0) == 0
