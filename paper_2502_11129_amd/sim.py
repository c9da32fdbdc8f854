"""Thin ctypes binding of libsim.so (the C ABI declared in include/sim.h).

Argument marshalling only: every simulation step runs in the HIP kernels of
libsim.so.  PyTorch provides the device workspace and the stream.  If the
library has not been built, importing works but creating a Simulator raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsim.so")
_lib = None

SIM_OK, SIM_E_INVALID, SIM_E_NOMEM, SIM_E_DEVICE, SIM_E_STATE, SIM_E_HOST = 0, -1, -2, -3, -4, -5
SIM_ROOT_FREE, SIM_ROOT_FIXED = 0, 1
SIM_HOST, SIM_DEVICE = 0, 1
EXPORTED = ("sim_create", "sim_workspace_bytes", "sim_bind", "sim_step_batch", "sim_rollout", "sim_fitness",
            "sim_get_state", "sim_set_state", "sim_counters", "sim_rollout_split", "sim_rollout_host", "sim_bins",
            "sim_variant_bins", "sim_bin_factorization", "sim_chunk_plan", "sim_launch_times", "sim_kernel_variants", "sim_split_allocation", "sim_plan_split", "sim_destroy", "sim_last_error")

_F = C.POINTER(C.c_float)
_I32 = C.POINTER(C.c_int32)


class sim_model_desc(C.Structure):
    _fields_ = [("n_variants", C.c_int32), ("root_type", C.c_int32), ("body_offset", _I32), ("parent", _I32),
                ("half_ext", _F), ("mass", _F), ("anchor_parent", _F), ("anchor_child", _F), ("rest_quat", _F),
                ("axis", _F), ("cpg", _F), ("mu", _F), ("q0", _F), ("v0", _F), ("root_pose", _F),
                ("kp", C.c_float), ("kd", C.c_float), ("tau_max", C.c_float), ("k_contact", C.c_float),
                ("b_contact", C.c_float), ("dt", C.c_float), ("gravity", C.c_float * 3), ("pgs_iters", C.c_int32),
                ("ball", _F), ("self_collision", C.c_int32)]


class sim_options(C.Structure):
    _fields_ = [("contacts_in_registers", C.c_int32), ("use_graph", C.c_int32), ("steps_per_launch", C.c_int32),
                ("streams", C.c_int32), ("min_body_slots", C.c_int32), ("ncr_by_nvc", C.c_int32 * 6),
                ("time_launches", C.c_int32), ("single_launch", C.c_int32), ("host_factorization", C.c_int32),
                ("min_nv_capacity", C.c_int32), ("slots32_min_nvc", C.c_int32), ("gpu_factorization", C.c_int32),
                ("host_fault_items", C.c_int32)]


NVC_CAPS = (8, 12, 16, 20, 24, 28)
HOST_FACTORIZATIONS = ("dense", "tree")   # SIM_FACTOR_DENSE, SIM_FACTOR_TREE
GPU_FACTORIZATIONS = HOST_FACTORIZATIONS


def make_options(contacts_in_registers=0, use_graph=False, steps_per_launch=0, streams=0, min_body_slots=0,
                 ncr_by_nvc=None, time_launches=False, single_launch=False, host_factorization="dense",
                 min_nv_capacity=0, slots32_min_nvc=0, gpu_factorization="dense", host_fault_items=0):
    o = sim_options()
    o.contacts_in_registers = int(contacts_in_registers)
    o.use_graph = int(bool(use_graph))
    o.steps_per_launch = int(steps_per_launch)
    o.streams = int(streams)
    o.min_body_slots = int(min_body_slots)
    o.time_launches = int(bool(time_launches))
    o.single_launch = int(bool(single_launch))
    o.host_factorization = HOST_FACTORIZATIONS.index(host_factorization)
    o.min_nv_capacity = int(min_nv_capacity)
    o.slots32_min_nvc = int(slots32_min_nvc)
    o.gpu_factorization = GPU_FACTORIZATIONS.index(gpu_factorization)
    o.host_fault_items = int(host_fault_items)
    for nvc, v in (ncr_by_nvc or {}).items():
        o.ncr_by_nvc[NVC_CAPS.index(int(nvc))] = int(v)
    return o


class sim_split_plan(C.Structure):
    _fields_ = [("n_host_paper", C.c_int32), ("n_host_makespan", C.c_int32), ("makespan_paper_s", C.c_double),
                ("makespan_opt_s", C.c_double), ("host_s_per_variant", C.c_double), ("gpu_points", C.c_int32),
                ("reserved", C.c_int32), ("gpu_n", C.c_int32 * 8), ("gpu_s", C.c_double * 8)]


class sim_split_times(C.Structure):
    _fields_ = [("combined_s", C.c_double), ("gpu_s", C.c_double), ("host_s", C.c_double),
                ("n_gpu", C.c_int32), ("n_host", C.c_int32), ("host_threads", C.c_int32), ("n_requeued", C.c_int32)]


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load libsim.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2502_11129_amd.build`")
    # torch ships its own HIP runtime (same soname); load it first so the process
    # holds a single runtime that both torch and libsim use.
    import torch  # noqa: F401
    lib = C.CDLL(_LIB_PATH)
    P, I, VP, SZ = C.c_void_p, C.c_int, C.c_void_p, C.c_size_t
    lib.sim_create.argtypes = [C.POINTER(sim_model_desc), C.POINTER(sim_options), C.POINTER(P)]
    lib.sim_create.restype = I
    lib.sim_workspace_bytes.argtypes = [P, C.POINTER(SZ)]
    lib.sim_bind.argtypes = [P, VP, SZ, VP]
    lib.sim_step_batch.argtypes = [P, C.c_int32, VP]
    lib.sim_rollout.argtypes = [P, C.c_int32, VP]
    lib.sim_fitness.argtypes = [P, VP, I, VP]
    lib.sim_get_state.argtypes = [P, _F, _F, C.POINTER(C.c_int64), I, VP]
    lib.sim_set_state.argtypes = [P, _F, _F, C.POINTER(C.c_int64), I, VP]
    lib.sim_counters.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), I, VP]
    lib.sim_bins.argtypes = [P, _I32, _I32, C.c_int32]
    lib.sim_rollout_split.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, VP, C.POINTER(sim_split_times)]
    lib.sim_rollout_host.argtypes = [P, C.c_int32, C.c_int32, _F, C.POINTER(C.c_double)]
    lib.sim_kernel_variants.argtypes = [_I32, _I32, C.c_int32]
    lib.sim_launch_times.argtypes = [P, _I32, _F, _I32, C.c_int32]
    lib.sim_variant_bins.argtypes = [P, _I32]
    lib.sim_bin_factorization.argtypes = [P, _I32, _I32, C.c_int32]
    lib.sim_chunk_plan.argtypes = [P, SZ, _I32, _I32, C.c_int32]
    lib.sim_split_allocation.argtypes = [C.c_int32, _I32, C.POINTER(C.c_double), C.c_int32, C.c_double, _I32, _I32,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.sim_plan_split.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, VP, C.POINTER(sim_split_plan)]
    lib.sim_destroy.argtypes = [P]
    lib.sim_destroy.restype = None
    lib.sim_last_error.argtypes = [P]
    lib.sim_last_error.restype = C.c_char_p
    for name in ("sim_workspace_bytes", "sim_bind", "sim_step_batch", "sim_rollout", "sim_fitness",
                 "sim_get_state", "sim_set_state", "sim_counters", "sim_bins", "sim_rollout_split",
                 "sim_rollout_host", "sim_variant_bins", "sim_bin_factorization", "sim_chunk_plan", "sim_launch_times", "sim_kernel_variants", "sim_split_allocation", "sim_plan_split"):
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def make_desc(pop):
    """Build a sim_model_desc over the arrays of a Population (kept alive by the returned tuple)."""
    keep = dict(bo=np.ascontiguousarray(pop.body_offset, np.int32), parent=np.ascontiguousarray(pop.parent, np.int32),
                half=_f32(pop.half_ext), mass=_f32(pop.mass), ap=_f32(pop.anchor_parent), ac=_f32(pop.anchor_child),
                rq=_f32(pop.rest_quat), axis=_f32(pop.axis), cpg=_f32(pop.cpg), mu=_f32(pop.mu), q0=_f32(pop.q0),
                v0=_f32(pop.v0), rp=_f32(pop.root_pose),
                ball=None if getattr(pop, "ball", None) is None else _f32(pop.ball))
    p = pop.params
    f = lambda a: a.ctypes.data_as(_F)
    d = sim_model_desc()
    d.n_variants = int(keep["bo"].shape[0] - 1)
    d.root_type = int(pop.root_type)
    d.body_offset = keep["bo"].ctypes.data_as(_I32)
    d.parent = keep["parent"].ctypes.data_as(_I32)
    d.half_ext, d.mass, d.anchor_parent, d.anchor_child = f(keep["half"]), f(keep["mass"]), f(keep["ap"]), f(keep["ac"])
    d.rest_quat, d.axis, d.cpg, d.mu = f(keep["rq"]), f(keep["axis"]), f(keep["cpg"]), f(keep["mu"])
    d.q0, d.v0, d.root_pose = f(keep["q0"]), f(keep["v0"]), f(keep["rp"])
    d.kp, d.kd, d.tau_max = p["kp"], p["kd"], p["tau_max"]
    d.k_contact, d.b_contact, d.dt = p["k_contact"], p["b_contact"], p["dt"]
    d.gravity[0], d.gravity[1], d.gravity[2] = p["gravity"]
    d.pgs_iters = int(p["pgs_iters"])
    d.ball = f(keep["ball"]) if keep["ball"] is not None else None
    d.self_collision = int(bool(getattr(pop, "self_collision", False)))
    return d, keep


def kernel_variants(ball=False, self_collision=False):
    """Compiled kernels as (nv capacity, body capacity, contacts in registers)
    of the plane-only family, the family whose variants carry a ball
    (ball=True) or the self-collision family (self_collision=True)."""
    lib = load()
    n = C.c_int32()
    info = np.zeros(5 * 64, np.int32)
    assert lib.sim_kernel_variants(C.byref(n), info.ctypes.data_as(_I32), 64) == SIM_OK
    rows = [tuple(int(x) for x in info[5 * i:5 * i + 5]) for i in range(n.value)]
    return [r[:3] for r in rows if r[3] == int(bool(ball)) and r[4] == int(bool(self_collision))]


def split_allocation(n, gpu_n, gpu_s, host_s_per_variant):
    """The C ABI's allocation rule on measured curves; returns a dict."""
    lib = load()
    gn = np.ascontiguousarray(gpu_n, np.int32)
    gs = np.ascontiguousarray(gpu_s, np.float64)
    hp, hm = C.c_int32(), C.c_int32()
    mp, mo = C.c_double(), C.c_double()
    rc = lib.sim_split_allocation(int(n), gn.ctypes.data_as(_I32), gs.ctypes.data_as(C.POINTER(C.c_double)),
                                  len(gn), float(host_s_per_variant), C.byref(hp), C.byref(hm), C.byref(mp),
                                  C.byref(mo))
    if rc != SIM_OK:
        raise SimError(rc, lib.sim_last_error(None).decode())
    return dict(n_host_paper=hp.value, n_host_makespan=hm.value, makespan_paper_s=mp.value,
                makespan_opt_s=mo.value)


class Handle:
    """Host-only handle (sim_create): validation and packing, no device work.
    Keyword options are those of sim_options (see make_options)."""

    def __init__(self, pop, contacts_in_registers: int = 0, use_graph: bool = False, **options):
        self.lib = load()
        self.pop = pop
        desc, self._keep = make_desc(pop)
        opts = make_options(contacts_in_registers, use_graph, **options)
        self.options = dict(contacts_in_registers=contacts_in_registers, use_graph=use_graph, **options)
        h = C.c_void_p()
        rc = self.lib.sim_create(C.byref(desc), C.byref(opts), C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, self.lib.sim_last_error(None).decode())
        self.h = h
        self.n = desc.n_variants
        self.nq = np.asarray(pop.nq)
        self.nv = np.asarray(pop.nv)

    def _check(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, self.lib.sim_last_error(self.h).decode())

    def workspace_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self.lib.sim_workspace_bytes(self.h, C.byref(b)))
        return int(b.value)

    def bins(self):
        n = C.c_int32()
        info = np.zeros(4 * 64, np.int32)
        self._check(self.lib.sim_bins(self.h, C.byref(n), info.ctypes.data_as(_I32), 64))
        return [tuple(int(x) for x in info[4 * i:4 * i + 4]) for i in range(n.value)]

    def bin_factorization(self):
        """Per bin (sim_bins order): "dense" or "tree", the kernel's factorisation of M~."""
        n = C.c_int32()
        f = np.zeros(64, np.int32)
        self._check(self.lib.sim_bin_factorization(self.h, C.byref(n), f.ctypes.data_as(_I32), 64))
        return [GPU_FACTORIZATIONS[int(x)] for x in f[:n.value]]

    def chunk_plan(self, max_workspace_bytes: int):
        """Ends of consecutive chunks (user order) whose handles each fit the workspace cap."""
        n = C.c_int32()
        rc = self.lib.sim_chunk_plan(self.h, int(max_workspace_bytes), C.byref(n), None, 0)
        if rc not in (SIM_OK, SIM_E_INVALID) or (rc == SIM_E_INVALID and n.value == 0):
            self._check(rc)
        ends = np.zeros(max(n.value, 1), np.int32)
        self._check(self.lib.sim_chunk_plan(self.h, int(max_workspace_bytes), C.byref(n), ends.ctypes.data_as(_I32),
                                            len(ends)))
        return ends[:n.value].tolist()

    def variant_bins(self):
        out = np.zeros(self.n, np.int32)
        self._check(self.lib.sim_variant_bins(self.h, out.ctypes.data_as(_I32)))
        return out

    def rollout_host(self, T: int, threads: int = 1):
        """Every variant on host threads (no device work); returns (fitness, seconds)."""
        fit = np.zeros(self.n, np.float32)
        sec = C.c_double()
        self._check(self.lib.sim_rollout_host(self.h, int(T), int(threads), fit.ctypes.data_as(_F), C.byref(sec)))
        return fit, sec.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Simulator(Handle):
    """A bound simulator: workspace allocated by torch on the current device."""

    def __init__(self, pop, contacts_in_registers: int = 0, use_graph: bool = False, device=None, **options):
        import torch
        super().__init__(pop, contacts_in_registers, use_graph, **options)
        self.torch = torch
        self.device = torch.device("cuda" if device is None else device)
        self.ws = torch.empty(max(self.workspace_bytes(), 256), dtype=torch.uint8, device=self.device)
        self._check(self.lib.sim_bind(self.h, C.c_void_p(self.ws.data_ptr()), self.ws.numel(), self.stream()))

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def step(self, n: int = 1):
        self._check(self.lib.sim_step_batch(self.h, int(n), self.stream()))

    def rollout(self, T: int):
        self._check(self.lib.sim_rollout(self.h, int(T), self.stream()))

    def fitness(self) -> np.ndarray:
        out = np.zeros(self.n, np.float32)
        self._check(self.lib.sim_fitness(self.h, C.c_void_p(out.ctypes.data), SIM_HOST, self.stream()))
        return out

    def fitness_device(self, out=None):
        if out is None:
            out = self.torch.empty(self.n, dtype=self.torch.float32, device=self.device)
        self._check(self.lib.sim_fitness(self.h, C.c_void_p(out.data_ptr()), SIM_DEVICE, self.stream()))
        return out

    def get_state(self):
        q = np.zeros(int(self.nq.sum()), np.float32)
        v = np.zeros(int(self.nv.sum()), np.float32)
        k = np.zeros(self.n, np.int64)
        self._check(self.lib.sim_get_state(self.h, q.ctypes.data_as(_F), v.ctypes.data_as(_F),
                                           k.ctypes.data_as(C.POINTER(C.c_int64)), SIM_HOST, self.stream()))
        return q, v, k

    def set_state(self, q, v, k=None):
        q = _f32(q)
        v = _f32(v)
        kk = None if k is None else np.ascontiguousarray(k, np.int64)
        self._check(self.lib.sim_set_state(self.h, q.ctypes.data_as(_F), v.ctypes.data_as(_F),
                                           None if kk is None else kk.ctypes.data_as(C.POINTER(C.c_int64)),
                                           SIM_HOST, self.stream()))

    def get_state_device(self, q=None, v=None, k=None):
        """State into device tensors (variant-CSR layout, stream-ordered, no sync)."""
        t = self.torch
        q = t.empty(int(self.nq.sum()), dtype=t.float32, device=self.device) if q is None else q
        v = t.empty(int(self.nv.sum()), dtype=t.float32, device=self.device) if v is None else v
        k = t.empty(self.n, dtype=t.int64, device=self.device) if k is None else k
        self._check(self.lib.sim_get_state(self.h, C.cast(q.data_ptr(), _F), C.cast(v.data_ptr(), _F),
                                           C.cast(k.data_ptr(), C.POINTER(C.c_int64)), SIM_DEVICE, self.stream()))
        return q, v, k

    def set_state_device(self, q, v, k=None):
        """State from device tensors (variant-CSR layout); k may be None (kept)."""
        self._check(self.lib.sim_set_state(self.h, C.cast(q.data_ptr(), _F), C.cast(v.data_ptr(), _F),
                                           None if k is None else C.cast(k.data_ptr(), C.POINTER(C.c_int64)),
                                           SIM_DEVICE, self.stream()))

    def counters_device(self):
        """Counters into device tensors: (rows_contact u64 as int64, rows_clamp, status as int32)."""
        t = self.torch
        a = t.empty(self.n, dtype=t.int64, device=self.device)
        b = t.empty(self.n, dtype=t.int64, device=self.device)
        s = t.empty(self.n, dtype=t.int32, device=self.device)
        self._check(self.lib.sim_counters(self.h, C.cast(a.data_ptr(), C.POINTER(C.c_uint64)),
                                          C.cast(b.data_ptr(), C.POINTER(C.c_uint64)),
                                          C.cast(s.data_ptr(), C.POINTER(C.c_uint32)), SIM_DEVICE, self.stream()))
        return a, b, s

    def rollout_split(self, T: int, n_host: int, threads: int):
        """Concurrent GPU + host-thread rollout; returns the timing record as a dict."""
        t = sim_split_times()
        self._check(self.lib.sim_rollout_split(self.h, int(T), int(n_host), int(threads), self.stream(), C.byref(t)))
        return dict(combined_s=t.combined_s, gpu_s=t.gpu_s, host_s=t.host_s, n_gpu=t.n_gpu, n_host=t.n_host,
                    host_threads=t.host_threads, n_requeued=t.n_requeued)

    def launch_times(self):
        """Per bin (sim_bins order): (milliseconds of its launches, number of launches) of the last run."""
        n = C.c_int32()
        ms = np.zeros(64, np.float32)
        cnt = np.zeros(64, np.int32)
        self._check(self.lib.sim_launch_times(self.h, C.byref(n), ms.ctypes.data_as(_F), cnt.ctypes.data_as(_I32), 64))
        return [(float(ms[i]), int(cnt[i])) for i in range(n.value)]

    def plan_split(self, T_pilot: int, threads: int, host_sample: int):
        """Pilot measurements and the two allocations (paper rule, makespan rule)."""
        p = sim_split_plan()
        self._check(self.lib.sim_plan_split(self.h, int(T_pilot), int(threads), int(host_sample), self.stream(),
                                            C.byref(p)))
        k = p.gpu_points
        return dict(n_host_paper=p.n_host_paper, n_host_makespan=p.n_host_makespan,
                    makespan_paper_s=p.makespan_paper_s, makespan_opt_s=p.makespan_opt_s,
                    host_s_per_variant=p.host_s_per_variant, gpu_n=list(p.gpu_n[:k]), gpu_s=list(p.gpu_s[:k]))

    def counters(self):
        a = np.zeros(self.n, np.uint64)
        b = np.zeros(self.n, np.uint64)
        s = np.zeros(self.n, np.uint32)
        self._check(self.lib.sim_counters(self.h, a.ctypes.data_as(C.POINTER(C.c_uint64)),
                                          b.ctypes.data_as(C.POINTER(C.c_uint64)),
                                          s.ctypes.data_as(C.POINTER(C.c_uint32)), SIM_HOST, self.stream()))
        return a, b, s


def rollout_in_chunks(pop, T: int, max_workspace_bytes=None, device=None, **options):
    """Rollout of T steps for a population of any size: consecutive chunks
    (sim_chunk_plan) whose workspaces each fit max_workspace_bytes (default:
    90 % of the device memory free now) are created, bound and run one after
    another.  Returns dict(fitness, rows_contact, rows_clamp, status, chunks)
    in user order; per-variant results equal those of one handle over the
    whole population."""
    import torch
    dev = torch.device("cuda" if device is None else device)
    if max_workspace_bytes is None:
        free, _ = torch.cuda.mem_get_info(dev)
        max_workspace_bytes = int(0.9 * free)
    probe = Handle(pop, **options)
    ends = probe.chunk_plan(max_workspace_bytes)
    probe.close()
    n = pop.n_variants
    fit = np.zeros(n, np.float32)
    rc, rl = np.zeros(n, np.uint64), np.zeros(n, np.uint64)
    st = np.zeros(n, np.uint32)
    start = 0
    for e in ends:
        sim = Simulator(pop.subset(np.arange(start, e)), device=dev, **options)
        sim.rollout(T)
        fit[start:e] = sim.fitness()
        rc[start:e], rl[start:e], st[start:e] = sim.counters()
        sim.close()
        del sim
        start = e
    return dict(fitness=fit, rows_contact=rc, rows_clamp=rl, status=st, chunks=ends)
