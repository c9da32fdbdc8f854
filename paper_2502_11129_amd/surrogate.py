"""Thin ctypes binding of the surrogate C ABI (include/sur.h) in libsim.so,
plus the host-side orchestration of training and screening.

Argument marshalling and call order only: features, forward and backward
passes, Adam, target standardisation and top-k selection all run in the HIP
kernels of libsim.so; torch supplies device memory and the stream.  Random
draws (initial weights, epoch permutations, candidate genotypes) come from
the seeded input generators and are passed in.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import sim as _sim
from . import workloads as W

SUR_N_PARAMS = 164865
SUR_N_FEAT = 128
EXPORTED = ("sur_create", "sur_workspace_bytes", "sur_bind", "sur_features", "sur_predict", "sur_train_step",
            "sur_train_epoch", "sur_adam_step", "sur_get_grad", "sur_get_state", "sur_set_state", "sur_topk",
            "sur_standardize", "sur_destroy", "sur_last_error", "sur_topk_noalloc")
SUR_TOPK_NOALLOC_MAX = 1 << 24

_F = C.POINTER(C.c_float)


class sur_config(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("reserved", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


class SurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = _sim.load()
    P, I, VP = C.c_void_p, C.c_int, C.c_void_p
    lib.sur_create.argtypes = [C.POINTER(sur_config), C.POINTER(P)]
    lib.sur_workspace_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
    lib.sur_bind.argtypes = [P, VP, C.c_size_t, _F, VP]
    lib.sur_features.argtypes = [P, C.c_int64, VP, VP, VP, VP, VP, VP, VP]
    lib.sur_predict.argtypes = [P, C.c_int64, VP, C.c_int64, VP, VP, VP]
    lib.sur_train_step.argtypes = [P, C.c_int32, VP, C.c_int64, VP, VP, VP, VP]
    lib.sur_train_epoch.argtypes = [P, C.c_int64, VP, C.c_int64, VP, VP, C.c_int32, VP, VP]
    lib.sur_adam_step.argtypes = [P, VP, VP]
    lib.sur_get_grad.argtypes = [P, VP, I, VP]
    lib.sur_get_state.argtypes = [P, _F, _F, _F, C.POINTER(C.c_int64), VP]
    lib.sur_set_state.argtypes = [P, _F, _F, _F, C.c_int64, VP]
    lib.sur_topk.argtypes = [P, C.c_int64, VP, C.c_int64, VP, VP]
    lib.sur_topk_noalloc.argtypes = [C.c_int64, VP, C.c_int64, VP, VP, C.c_char_p, C.c_size_t]
    lib.sur_standardize.argtypes = [P, C.c_int64, VP, VP, C.POINTER(C.c_double), VP]
    lib.sur_destroy.argtypes = [P]
    lib.sur_destroy.restype = None
    lib.sur_last_error.argtypes = [P]
    lib.sur_last_error.restype = C.c_char_p
    for n in EXPORTED:
        if n not in ("sur_destroy", "sur_last_error"):
            getattr(lib, n).restype = I
    _lib = lib
    return lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def topk_noalloc(scores, k, out=None, stream=None):
    """sur_topk_noalloc: indices of the k largest of the device float32 tensor
    `scores` (ascending index order), with the library's static scratch and no
    allocation inside the call; `out` (device int32 [k]) may be passed so that
    nothing at all is allocated.  Raises SurError on a refused size."""
    import torch
    lib = load()
    if out is None:
        out = torch.empty(int(k), dtype=torch.int32, device=scores.device)
    if stream is None:
        stream = torch.cuda.current_stream(scores.device).cuda_stream
    err = C.create_string_buffer(256)
    rc = lib.sur_topk_noalloc(int(scores.shape[0]), _ptr(scores), int(k), _ptr(out), C.c_void_p(stream), err, 256)
    if rc != 0:
        raise SurError(rc, err.value.decode())
    return out


class Surrogate:
    """A bound surrogate network on the current torch device."""

    def __init__(self, params=None, seed=0, max_batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, device=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda" if device is None else device)
        cfg = sur_config(int(max_batch), 0, float(lr), float(beta1), float(beta2), float(eps))
        h = C.c_void_p()
        rc = self.lib.sur_create(C.byref(cfg), C.byref(h))
        if rc:
            raise SurError(rc, self.lib.sur_last_error(None).decode())
        self.h = h
        self.max_batch = int(max_batch)
        b = C.c_size_t()
        self._check(self.lib.sur_workspace_bytes(self.h, C.byref(b)))
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        p0 = np.ascontiguousarray(W.mlp_init(seed) if params is None else params, np.float32)
        assert p0.shape == (SUR_N_PARAMS,)
        self._check(self.lib.sur_bind(self.h, _ptr(self.ws), self.ws.numel(), p0.ctypes.data_as(_F), self.stream()))

    def _check(self, rc):
        if rc:
            raise SurError(rc, self.lib.sur_last_error(self.h).decode())

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    # -- data
    def upload_genotypes(self, g):
        a = W.genotype_arrays(g)
        return {k: self.torch.from_numpy(v).to(self.device) for k, v in a.items()}

    def features(self, gd, n=None):
        """Device genotype arrays (upload_genotypes) -> BF16 features [n, 128]."""
        n = int(gd["nh"].shape[0]) if n is None else int(n)
        X = self.torch.empty((n, SUR_N_FEAT), dtype=self.torch.bfloat16, device=self.device)
        self._check(self.lib.sur_features(self.h, n, _ptr(gd["nh"]), _ptr(gd["parent"]), _ptr(gd["face"]),
                                          _ptr(gd["axis"]), _ptr(gd["cpg"]), _ptr(X), self.stream()))
        return X

    # -- network
    def predict(self, X, idx=None, out=None):
        n = int(X.shape[0]) if idx is None else int(idx.shape[0])
        if out is None:
            out = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.sur_predict(self.h, n, _ptr(X), int(X.shape[0]), _ptr(idx), _ptr(out), self.stream()))
        return out

    def train_step(self, X, target, idx):
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.sur_train_step(self.h, int(idx.shape[0]), _ptr(X), int(X.shape[0]), _ptr(target),
                                            _ptr(idx), _ptr(loss), self.stream()))
        return loss

    def train_epoch(self, X, target, perm, batch=4096):
        n = int(perm.shape[0])
        losses = self.torch.empty(-(-n // batch), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.sur_train_epoch(self.h, n, _ptr(X), int(X.shape[0]), _ptr(target), _ptr(perm),
                                             int(batch), _ptr(losses), self.stream()))
        return losses

    def adam_step(self, grad):
        self._check(self.lib.sur_adam_step(self.h, _ptr(grad), self.stream()))

    def grad(self):
        out = np.zeros(SUR_N_PARAMS, np.float32)
        self._check(self.lib.sur_get_grad(self.h, C.c_void_p(out.ctypes.data), 0, self.stream()))
        return out

    def get_state(self):
        p, m, v = (np.zeros(SUR_N_PARAMS, np.float32) for _ in range(3))
        t = C.c_int64()
        self._check(self.lib.sur_get_state(self.h, p.ctypes.data_as(_F), m.ctypes.data_as(_F), v.ctypes.data_as(_F),
                                           C.byref(t), self.stream()))
        return p, m, v, int(t.value)

    def set_state(self, params, m=None, v=None, t=0):
        keep = [None if a is None else np.ascontiguousarray(a, np.float32) for a in (params, m, v)]
        ptrs = [None if a is None else a.ctypes.data_as(_F) for a in keep]
        self._check(self.lib.sur_set_state(self.h, ptrs[0], ptrs[1], ptrs[2], int(t), self.stream()))

    # -- selection
    def topk(self, scores, k):
        out = self.torch.empty(int(k), dtype=self.torch.int32, device=self.device)
        self._check(self.lib.sur_topk(self.h, int(scores.shape[0]), _ptr(scores), int(k), _ptr(out), self.stream()))
        return out

    def standardize(self, y, out=None):
        if out is None:
            out = self.torch.empty_like(y)
        st = (C.c_double * 2)()
        self._check(self.lib.sur_standardize(self.h, int(y.shape[0]), _ptr(y), _ptr(out), st, self.stream()))
        return out, float(st[0]), float(st[1])

    def close(self):
        if getattr(self, "h", None):
            self.lib.sur_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


# ----------------------------------------------------------------------------- orchestration
def simulate_fitness(g, T=5000, chunk=32768, device=None, nudge=None):
    """Exact fitness of genotypes g (the simulator is the judge): rollouts of
    T steps in chunks of `chunk` robots; with nudge = seed, from initial
    positions moved by one float32 ulp (workloads.nudged).  Returns (fitness
    float32 [n], GPU seconds of the rollouts, host seconds spent building
    models)."""
    import torch
    out = np.zeros(len(g), np.float32)
    gpu_s = host_s = 0.0
    for c0 in range(0, len(g), chunk):
        t0 = time.perf_counter()
        pop = W.population_from_genotypes(g.take(np.arange(c0, min(len(g), c0 + chunk))), steps=T)
        if nudge is not None:
            pop = W.nudged(pop, nudge * 1000003 + c0)
        sim = _sim.Simulator(pop, device=device)
        host_s += time.perf_counter() - t0
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        sim.rollout(T)
        e1.record(st)
        out[c0:c0 + pop.n_variants] = sim.fitness()
        gpu_s += e0.elapsed_time(e1) / 1e3
        sim.close()
        del sim
    return out, gpu_s, host_s


def train(sur, X, y_std, epochs, batch=4096, seed=0):
    """Train on rows of X (device BF16) against standardised targets y_std
    (device float); epoch permutations from rng([6, seed, epoch]).  Returns the
    per-batch losses as a host array [epochs, batches]."""
    torch = sur.torch
    n = int(X.shape[0])
    losses = []
    for e in range(epochs):
        perm = np.random.default_rng([6, seed, e]).permutation(n).astype(np.int32)
        perm_d = torch.from_numpy(perm).to(sur.device)
        losses.append(sur.train_epoch(X, y_std, perm_d, batch))
    return torch.stack(losses).cpu().numpy()


def screen(sur, gd, n, k):
    """Features -> predictions -> indices of the k best predictions, all on the
    device; returns (indices int32 [k] ascending, predictions, seconds by stage)."""
    torch = sur.torch
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(st)
    X = sur.features(gd, n)
    ev[1].record(st)
    pred = sur.predict(X)
    ev[2].record(st)
    top = sur.topk(pred, k)
    ev[3].record(st)
    torch.cuda.synchronize()
    t = [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(3)]
    return top, pred, dict(features_s=t[0], predict_s=t[1], topk_s=t[2])
