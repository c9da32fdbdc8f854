"""Build libsim.so (HIP kernels for gfx950 + the C-ABI host library) in-tree.

Usage: python -m paper_2502_11129_amd.build  (or build() from Python).
The kernel translation units compile in parallel; objects go to _build/.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import json
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(os.path.dirname(PKG), "_build")
LIB = os.path.join(PKG, "libsim.so")
ARCH = os.environ.get("SIM_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM_INC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
API_INC = os.path.join(os.path.dirname(PKG), "include")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wno-unused-result"]
# Packed FP32 instructions stay disabled in every HIP translation unit; a * b + c
# is fused only within one expression, so every kernel variant (whatever its
# register budget or inlining context) rounds the same way.
DEVICE = [f"--offload-arch={ARCH}", "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _sources(csrc: str = CSRC):
    kern = sorted(glob.glob(os.path.join(csrc, "kernels", "*.hip")))
    host = [os.path.join(csrc, n) for n in ("kernel_registry.cpp", "sim_host.cpp", "host_worker.cpp", "sur_host.cpp",
                                         "ea_host.cpp")]
    return kern, host


RESOURCES = "kernel_resources.json"   # per-kernel registers, scratch, occupancy and LDS of the last build


def _resources(stderr: str) -> dict:
    """The compiler's kernel resource remarks (-Rpass-analysis=kernel-resource-usage)
    as {kernel: {field: value}}."""
    out, name = {}, None
    for line in stderr.splitlines():
        if "remark:" not in line or "kernel-resource-usage" not in line:
            continue
        text = line.split("remark:", 1)[1].split(" [-Rpass", 1)[0].strip()
        key, _, val = text.partition(":")
        key, val = key.strip(), val.strip()
        if key == "Function Name":
            name = val
            out[name] = {}
        elif name is not None:
            out[name][key] = int(val) if val.lstrip("-").isdigit() else val
    return out


def _compile(src: str, device: bool, csrc: str = CSRC, objdir: str = BUILD) -> tuple[str, dict]:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *(DEVICE if device else []), "-Rpass-analysis=kernel-resource-usage", "-I", csrc, "-c",
           src, "-o", obj]
    if not device:
        cmd = [HIPCC, *COMMON, "-I", csrc, "-I", API_INC, "-I", ROCM_INC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, (_resources(r.stderr) if device else {})


def build(jobs: int | None = None, verbose: bool = False, csrc: str = CSRC, lib: str = LIB, objdir: str = BUILD) -> str:
    """Compile every HIP source for gfx950 and link libsim.so (always rebuilds).
    csrc / lib / objdir: another source tree, library path and object folder
    (the per-phase profiling build uses an instrumented copy)."""
    os.makedirs(objdir, exist_ok=True)
    kern, host = _sources(csrc)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_compile, s, True, csrc, objdir) for s in kern] + \
            [ex.submit(_compile, s, False, csrc, objdir) for s in host]
        done = [f.result() for f in futs]
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(os.path.join(objdir, RESOURCES), "w") as f:
        json.dump(res, f, indent=0, sort_keys=True)
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


def build_host_sanitized(out_dir: str) -> str:
    """libsim.so with its host code (C ABI, packing, host worker, split and
    chunk planning) built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host pass only, -O1 -g) and the kernel objects of the last build():
    for host-only runs in a process that preloads the compiler's ASan runtime
    (asan_runtime()).  Returns the library path."""
    os.makedirs(out_dir, exist_ok=True)
    kern, host = _sources()
    kobjs = [os.path.join(BUILD, os.path.basename(k) + ".o") for k in kern]
    missing = [o for o in kobjs if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError(f"kernel objects missing (run build() first): {missing[:3]}")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    objs = []
    for src in host:
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC", "-Wno-unused-result", *san,
               "-I", CSRC, "-I", API_INC, "-I", ROCM_INC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        objs.append(obj)
    lib = os.path.join(out_dir, "libsim.so")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *san, *objs, *kobjs, "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return lib


def asan_runtime() -> str:
    """The ASan runtime of the compiler that build_host_sanitized() uses."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    return subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
