"""AddressSanitizer + UndefinedBehaviorSanitizer over the host C++: the FP64
oracle (g++) and the host side of the simulator library (C ABI, packing,
host worker, split and chunk planning; clang's host pass, the kernels
unchanged).  Each runs in a subprocess with the sanitizer runtime preloaded;
any finding aborts it.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitizer_driver.py")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(args, preload, timeout):
    env = dict(ENV, LD_PRELOAD=preload)
    r = subprocess.run([sys.executable, DRIVER, *args], env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0 and "clean" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    from oracle import oracle as O
    out = _run(["oracle", str(tmp_path)], O.asan_runtime(), 600)
    assert out.count("steps") == 6


def test_host_library_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_2502_11129_amd import build as B
    try:
        lib = B.build_host_sanitized(str(tmp_path))
    except FileNotFoundError as e:
        pytest.skip(f"no kernel objects to link against: {e}")
    out = _run(["sim", lib], B.asan_runtime(), 600)
    assert "failure and validation paths" in out
