"""Python binding of the peak probes (include/probe.h).

Argument marshalling only: torch supplies the device buffers and the stream;
the microbenchmarks run in the HIP library.
"""
from __future__ import annotations

import ctypes as C

from . import sim as _sim

EXPORTED = ("probe_fp32_fma", "probe_bf16_mfma", "probe_copy", "probe_sincos", "probe_last_error")
_lib = None


class ProbeError(RuntimeError):
    pass


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _sim.load()
    VP, I32, D = C.c_void_p, C.c_int32, C.POINTER(C.c_double)
    lib.probe_fp32_fma.argtypes = [VP, I32, I32, VP, D]
    lib.probe_bf16_mfma.argtypes = [VP, I32, I32, VP, D]
    lib.probe_copy.argtypes = [VP, VP, C.c_size_t, VP, D]
    lib.probe_sincos.argtypes = [VP, VP, VP, C.c_int64, VP]
    for n in ("probe_fp32_fma", "probe_bf16_mfma", "probe_copy", "probe_sincos"):
        getattr(lib, n).restype = C.c_int
    lib.probe_last_error.argtypes = []
    lib.probe_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc:
        raise ProbeError(f"{load().probe_last_error().decode()} (code {rc})")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def fp32_fma(blocks=8192, iters=1024, reps=3):
    """Best of `reps` FP32 FMA probe launches, TFLOP/s."""
    import torch
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    best = 0.0
    for _ in range(reps):
        r = C.c_double()
        _check(load().probe_fp32_fma(C.c_void_p(sink.data_ptr()), blocks, iters, _stream(), C.byref(r)))
        best = max(best, r.value)
    return best


def bf16_mfma(blocks=8192, iters=512, reps=3):
    """Best of `reps` BF16 MFMA probe launches, TFLOP/s."""
    import torch
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    best = 0.0
    for _ in range(reps):
        r = C.c_double()
        _check(load().probe_bf16_mfma(C.c_void_p(sink.data_ptr()), blocks, iters, _stream(), C.byref(r)))
        best = max(best, r.value)
    return best


def copy(nbytes=1 << 30, reps=3):
    """Best of `reps` device copies of nbytes, GB/s (read + written)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = 0.0
    for _ in range(reps):
        r = C.c_double()
        _check(load().probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, _stream(),
                                 C.byref(r)))
        best = max(best, r.value)
    ok = bool(torch.equal(src, dst))
    del src, dst
    if not ok:
        raise ProbeError("probe_copy: destination differs from source")
    return best


def sincos(x):
    """The rollout kernel's (sin x, cos x) for a float32 CUDA tensor x."""
    import torch
    x = x.contiguous()
    assert x.is_cuda and x.dtype == torch.float32
    sn, cs = torch.empty_like(x), torch.empty_like(x)
    _check(load().probe_sincos(C.c_void_p(x.data_ptr()), C.c_void_p(sn.data_ptr()), C.c_void_p(cs.data_ptr()),
                               x.numel(), _stream()))
    torch.cuda.synchronize()
    return sn, cs


def all_peaks():
    """Measured peaks of the running GPU as a dict (for roofline reports)."""
    return {"fp32_fma_tflops": fp32_fma(), "bf16_mfma_tflops": bf16_mfma(), "hbm_copy_GBs": copy()}
