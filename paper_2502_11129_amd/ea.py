"""Python binding of the evolutionary-loop kernels (include/ea.h).

Argument marshalling only: genotypes live on the device as dicts of torch
tensors in the layout of ``workloads.genotype_arrays`` (nh int32 [n],
parent/face/axis int8 [n, 20], cpg float32 [n, 20, 3]); every operator runs
in the HIP library, on torch's current stream.
"""
from __future__ import annotations

import ctypes as C

from . import sim as _sim

EXPORTED = ("ea_vary", "ea_tune_perturb", "ea_tune_accept", "ea_gather", "ea_last_error")
KEYS = ("nh", "parent", "face", "axis", "cpg")
_lib = None


class EaError(RuntimeError):
    pass


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _sim.load()
    VP, I32, U64 = C.c_void_p, C.c_int32, C.c_uint64
    lib.ea_vary.argtypes = [I32, VP, VP, VP, VP, VP, VP, I32, U64, I32, VP, VP, VP, VP, VP, VP]
    lib.ea_tune_perturb.argtypes = [I32, VP, VP, U64, I32, I32, VP, VP]
    lib.ea_tune_accept.argtypes = [I32, VP, VP, VP, VP, VP]
    lib.ea_gather.argtypes = [I32, VP, I32, VP, VP, VP, VP, VP, VP, I32, VP, VP, VP, VP, VP, VP,
                              VP, VP, VP, VP, VP, VP, VP]
    for n in ("ea_vary", "ea_tune_perturb", "ea_tune_accept", "ea_gather"):
        getattr(lib, n).restype = C.c_int
    lib.ea_last_error.argtypes = []
    lib.ea_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc):
    if rc:
        raise EaError(f"{load().ea_last_error().decode()} (code {rc})")


def empty_genotypes(n, device):
    import torch
    return dict(nh=torch.empty(n, dtype=torch.int32, device=device),
                parent=torch.empty((n, 20), dtype=torch.int8, device=device),
                face=torch.empty((n, 20), dtype=torch.int8, device=device),
                axis=torch.empty((n, 20), dtype=torch.int8, device=device),
                cpg=torch.empty((n, 20, 3), dtype=torch.float32, device=device))


def vary(parents, fitness, n_off, seed, generation):
    """n_off offspring of the parents (device dict) with the given fitness."""
    mu = int(parents["nh"].shape[0])
    out = empty_genotypes(int(n_off), parents["nh"].device)
    _check(load().ea_vary(mu, *(_p(parents[k]) for k in KEYS), _p(fitness), int(n_off), int(seed), int(generation),
                          *(_p(out[k]) for k in KEYS), _stream()))
    return out


def tune_perturb(geno, seed, generation, round_):
    """Lamarckian candidate controllers (cpg tensor) of the genotypes."""
    import torch
    n = int(geno["nh"].shape[0])
    cpg = torch.empty_like(geno["cpg"])
    _check(load().ea_tune_perturb(n, _p(geno["nh"]), _p(geno["cpg"]), int(seed), int(generation), int(round_),
                                  _p(cpg), _stream()))
    return cpg


def tune_accept(cpg_base, fit_base, cpg_cand, fit_cand):
    """In place: keep strictly better candidate controllers."""
    n = int(fit_base.shape[0])
    _check(load().ea_tune_accept(n, _p(cpg_base), _p(fit_base), _p(cpg_cand), _p(fit_cand), _stream()))


def gather(idx, a, fit_a=None, b=None, fit_b=None, with_fitness=True):
    """Rows idx of the concatenation [a; b] (device dicts); returns (dict, fitness or None)."""
    import torch
    k = int(idx.shape[0])
    dev = idx.device
    out = empty_genotypes(k, dev)
    fit_out = torch.empty(k, dtype=torch.float32, device=dev) if with_fitness else None
    n_a = int(a["nh"].shape[0])
    n_b = 0 if b is None else int(b["nh"].shape[0])
    bb = b if b is not None else {key: None for key in KEYS}
    _check(load().ea_gather(k, _p(idx), n_a, *(_p(a[key]) for key in KEYS), _p(fit_a), n_b,
                            *(_p(bb[key]) for key in KEYS), _p(fit_b), *(_p(out[key]) for key in KEYS),
                            _p(fit_out), _stream()))
    return out, fit_out
