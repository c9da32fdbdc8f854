"""ctypes wrapper of the FP64 reference simulator (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; the product path never loads it.

The wrapper accepts any object carrying the variant-CSR model arrays
(``body_offset``, ``parent``, ``half_ext``, ``mass``, ``anchor_parent``,
``anchor_child``, ``rest_quat``, ``axis``, ``cpg``, ``mu``, ``q0``, ``v0``,
``root_pose``, ``root_type``, ``params`` and optionally ``ball``: [N, 2] radius
and mass of one free sphere per variant, and ``self_collision``: contacts
between the boxes of one robot) -- the seeded generators produce
such objects; nothing here imports the HIP library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_native = {}


def _compile(out: str, native: bool) -> str:
    """g++ -O3 of oracle.cpp into ``out``; ``native`` adds -march=native (code
    for the CPU that compiles it, so only for the machine that runs it)."""
    tmp = out + ".tmp"
    arch = ["-march=native"] if native else []
    subprocess.check_call(["g++", "-O3", *arch, "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ -O3 (portable x86-64 code: the library
    travels to other machines with the tree, so no -march=native here)."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, native=False)
    return _LIB


def _declare(lib):
    P, I, D, F = C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_float)
    I32, I64, U32, U64 = (C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_uint32),
                          C.POINTER(C.c_uint64))
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [I, I32, I32, F, F, F, F, F, F, F, F, F, F, F, F, D, I, I, I, I]
    lib.orc_destroy.argtypes = [P]
    lib.orc_step.argtypes = [P, I, I]
    lib.orc_step_subset.argtypes = [P, I, I32, I, I]
    lib.orc_reset.argtypes = [P]
    lib.orc_rk4.argtypes = [P, I, I, I]
    lib.orc_fitness.argtypes = [P, D]
    lib.orc_get_state.argtypes = [P, D, D, I64, U32]
    lib.orc_set_state.argtypes = [P, D, D, I64]
    lib.orc_counters.argtypes = [P, U64, U64]
    lib.orc_plane_margin.argtypes = [P, D]
    lib.orc_invariants.argtypes = [P, I, D]
    lib.orc_fk.argtypes = [P, I, D, D, D, D, D]
    lib.orc_fk.restype = I
    lib.orc_dynamics.argtypes = [P, I, D, D, D, D]
    lib.orc_dynamics.restype = I
    lib.orc_contacts.argtypes = [P, I, D, I, I32, I32, D, D, D, D, I32]
    lib.orc_contacts.restype = I
    lib.orc_cholesky.argtypes = [I, D, D]
    lib.orc_cholesky.restype = I
    lib.orc_edge_contact.argtypes = [D, D, D, D, D, D, D, D, D]
    lib.orc_edge_contact.restype = I
    lib.orc_face_contacts.argtypes = [D, D, D, D, D, D, D, D, D, C.POINTER(C.c_int)]
    lib.orc_face_contacts.restype = I
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(C.CDLL(_LIB))
    return _lib


def load_native(directory: str):
    """The same source built -O3 -march=native into ``directory`` on the
    machine that calls this (for timing the oracle on that host's cores);
    compiled once per process and directory."""
    if directory not in _native:
        os.makedirs(directory, exist_ok=True)
        _native[directory] = _declare(C.CDLL(_compile(os.path.join(directory, "liboracle_native.so"), True)))
    return _native[directory]


def load_sanitized(directory: str):
    """The same source built with AddressSanitizer and UndefinedBehaviorSanitizer
    (-O1 -g, any finding aborts) into ``directory``.  Only loadable in a
    process started with the ASan runtime preloaded (``asan_runtime()``)."""
    key = ("asan", directory)
    if key not in _native:
        os.makedirs(directory, exist_ok=True)
        out = os.path.join(directory, "liboracle_asan.so")
        subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=undefined", "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC,
                               "-o", out])
        _native[key] = _declare(C.CDLL(out))
    return _native[key]


def asan_runtime() -> str:
    """Path of the compiler's ASan runtime (to preload for load_sanitized)."""
    return subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def cholesky(A: np.ndarray) -> np.ndarray:
    """The oracle's own textbook Cholesky (lower factor)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros_like(A)
    if _load().orc_cholesky(n, _p(A, C.c_double), _p(L, C.c_double)) != 0:
        raise np.linalg.LinAlgError("not positive definite")
    return L


def edge_contact(pP, RP, hP, pQ, RQ, hQ):
    """The oracle's edge-edge contact of two boxes P and Q (centre, 3x3
    rotation, half extents): (x, n, depth) with n pointing towards P, or None."""
    args = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (pP, RP, hP, pQ, RQ, hQ)]
    x, n, d = np.zeros(3), np.zeros(3), np.zeros(1)
    if not _load().orc_edge_contact(*[_p(a, C.c_double) for a in args], _p(x, C.c_double), _p(n, C.c_double),
                                    _p(d, C.c_double)):
        return None
    return x, n, float(d[0])


def face_contacts(pP, RP, hP, pQ, RQ, hQ):
    """The oracle's face contacts of two boxes P and Q (centre, 3x3 rotation,
    half extents): (points [m, 3], depths [m], n towards the points' box,
    'P' or 'Q' for the box the points belong to), m = 0 when there are none."""
    args = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in (pP, RP, hP, pQ, RQ, hQ)]
    x, d, n, inc = np.zeros(72), np.zeros(24), np.zeros(3), C.c_int(0)
    m = _load().orc_face_contacts(*[_p(a, C.c_double) for a in args], _p(x, C.c_double), _p(d, C.c_double),
                                  _p(n, C.c_double), C.byref(inc))
    return x[:3 * m].reshape(m, 3), d[:m], n, "Q" if inc.value else "P"


class Oracle:
    """Reference simulator over a population (FP64, or FP32 with precision=32).

    The model is the one a float32 simulator is handed: the per-body arrays
    and, unless ``float32_constants`` is False, the scalar constants (gains,
    contact law, time step, gravity) rounded to float32 and then computed
    with in FP64.  The time step matters most: the controller's clock
    t = k dt multiplies its rounding by k, so over 30 000 steps the float32
    and the decimal 0.002 s put the CPG clocks 3 microseconds apart.  The
    pins of the oracle itself pass False to take the constants exactly.
    ``lib`` selects another build of the same source (``load_native``)."""

    def __init__(self, pop, precision: int = 64, pgs_iters: int | None = None, params: dict | None = None,
                 float32_constants: bool = True, lib=None):
        lib = _load() if lib is None else lib
        prm = dict(pop.params)
        if params:
            prm.update(params)
        if float32_constants:
            for key in ("kp", "kd", "tau_max", "k_contact", "b_contact", "dt"):
                prm[key] = float(np.float32(prm[key]))
            prm["gravity"] = tuple(float(x) for x in np.asarray(prm["gravity"], np.float32))
        K = int(prm["pgs_iters"] if pgs_iters is None else pgs_iters)
        g = prm["gravity"]
        self._keep = dict(
            bo=np.ascontiguousarray(pop.body_offset, np.int32),
            parent=np.ascontiguousarray(pop.parent, np.int32),
            half=np.ascontiguousarray(pop.half_ext, np.float32),
            mass=np.ascontiguousarray(pop.mass, np.float32),
            ap=np.ascontiguousarray(pop.anchor_parent, np.float32),
            ac=np.ascontiguousarray(pop.anchor_child, np.float32),
            rq=np.ascontiguousarray(pop.rest_quat, np.float32),
            axis=np.ascontiguousarray(pop.axis, np.float32),
            cpg=np.ascontiguousarray(pop.cpg, np.float32),
            mu=np.ascontiguousarray(pop.mu, np.float32),
            q0=np.ascontiguousarray(pop.q0, np.float32),
            v0=np.ascontiguousarray(pop.v0, np.float32),
            rp=np.ascontiguousarray(pop.root_pose, np.float32),
            ball=(None if getattr(pop, "ball", None) is None else np.ascontiguousarray(pop.ball, np.float32)),
            prm=np.array([prm["kp"], prm["kd"], prm["tau_max"], prm["k_contact"], prm["b_contact"],
                          prm["dt"], g[0], g[1], g[2]], dtype=np.float64))
        k = self._keep
        self.n = int(k["bo"].shape[0] - 1)
        self.root_fixed = int(pop.root_type != 0)
        nb = np.diff(k["bo"]).astype(np.int64)
        self.has_ball = k["ball"] is not None
        self.nq = nb - 1 + (0 if self.root_fixed else 7) + (7 if self.has_ball else 0)
        self.nv = nb - 1 + (0 if self.root_fixed else 6) + (6 if self.has_ball else 0)
        self.q_off = np.concatenate([[0], np.cumsum(self.nq)])
        self.v_off = np.concatenate([[0], np.cumsum(self.nv)])
        self.dt = float(prm["dt"])
        self.precision = precision
        f = lambda a: _p(a, C.c_float)
        self.h = lib.orc_create(self.n, _p(k["bo"], C.c_int32), _p(k["parent"], C.c_int32), f(k["half"]),
                                f(k["mass"]), f(k["ap"]), f(k["ac"]), f(k["rq"]), f(k["axis"]), f(k["cpg"]),
                                f(k["mu"]), f(k["q0"]), f(k["v0"]), f(k["rp"]),
                                None if k["ball"] is None else f(k["ball"]), _p(k["prm"], C.c_double),
                                self.root_fixed, K, precision, int(bool(getattr(pop, "self_collision", False))))
        self._lib = lib

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.orc_destroy(self.h)
            self.h = None

    # -- whole-population operations --
    def step(self, n: int = 1, threads: int = 1):
        self._lib.orc_step(self.h, int(n), int(threads))

    def step_subset(self, idx, n: int = 1, threads: int = 1):
        idx = np.ascontiguousarray(idx, np.int32)
        self._lib.orc_step_subset(self.h, len(idx), _p(idx, C.c_int32), int(n), int(threads))

    def reset(self):
        self._lib.orc_reset(self.h)

    def rollout(self, T: int, threads: int = 1) -> np.ndarray:
        self.reset()
        self.step(T, threads)
        return self.fitness()

    def rk4(self, n: int = 1, pd: bool = False, threads: int = 1):
        self._lib.orc_rk4(self.h, int(n), int(pd), int(threads))

    def fitness(self) -> np.ndarray:
        out = np.zeros(self.n, np.float64)
        self._lib.orc_fitness(self.h, _p(out, C.c_double))
        return out

    def get_state(self):
        q = np.zeros(int(self.q_off[-1]), np.float64)
        v = np.zeros(int(self.v_off[-1]), np.float64)
        k = np.zeros(self.n, np.int64)
        s = np.zeros(self.n, np.uint32)
        self._lib.orc_get_state(self.h, _p(q, C.c_double), _p(v, C.c_double), _p(k, C.c_int64),
                                _p(s, C.c_uint32))
        return q, v, k, s

    def set_state(self, q, v, k=None):
        q = np.ascontiguousarray(q, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        kk = None if k is None else np.ascontiguousarray(k, np.int64)
        self._lib.orc_set_state(self.h, _p(q, C.c_double), _p(v, C.c_double),
                                None if kk is None else _p(kk, C.c_int64))

    def counters(self):
        a = np.zeros(self.n, np.uint64)
        b = np.zeros(self.n, np.uint64)
        self._lib.orc_counters(self.h, _p(a, C.c_uint64), _p(b, C.c_uint64))
        return a, b

    def plane_margin(self) -> np.ndarray:
        """Per variant, the smallest |height| above the plane of any box corner
        (and of the ball's lowest point) over the steps since the last reset or
        set_state: how close a contact came to switching on or off."""
        out = np.empty(self.n)
        self._lib.orc_plane_margin(self.h, _p(out, C.c_double))
        return out

    def invariants(self, vi: int = 0) -> np.ndarray:
        out = np.zeros(7, np.float64)
        self._lib.orc_invariants(self.h, int(vi), _p(out, C.c_double))
        return out

    # -- single-variant probes (FP64 handles) --
    def nbodies(self, vi: int) -> int:
        bo = self._keep["bo"]
        return int(bo[vi + 1] - bo[vi])

    def fk(self, vi: int, q):
        q = np.ascontiguousarray(q, np.float64)
        nb = self.nbodies(vi)
        R = np.zeros((nb, 3, 3)); p = np.zeros((nb, 3)); w = np.zeros((nb, 3)); o = np.zeros((nb, 3))
        assert self._lib.orc_fk(self.h, vi, _p(q, C.c_double), _p(R, C.c_double), _p(p, C.c_double),
                                _p(w, C.c_double), _p(o, C.c_double)) == 0
        return R, p, w, o

    def dynamics(self, vi: int, q, v):
        q = np.ascontiguousarray(q, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        nv = int(self.nv[vi])
        M = np.zeros((nv, nv)); c = np.zeros(nv)
        assert self._lib.orc_dynamics(self.h, vi, _p(q, C.c_double), _p(v, C.c_double),
                                      _p(M, C.c_double), _p(c, C.c_double)) == 0
        return M, c

    def contacts(self, vi: int, q, max_contacts: int = 256):
        q = np.ascontiguousarray(q, np.float64)
        nv = int(self.nv[vi])
        m = max_contacts
        body = np.zeros(m, np.int32); corner = np.zeros(m, np.int32)
        x = np.zeros((m, 3)); d = np.zeros(m); J = np.zeros((m, 3, nv)); nrm = np.zeros((m, 3))
        other = np.zeros(m, np.int32)
        n = self._lib.orc_contacts(self.h, vi, _p(q, C.c_double), m, _p(body, C.c_int32),
                                   _p(corner, C.c_int32), _p(x, C.c_double), _p(d, C.c_double),
                                   _p(J, C.c_double), _p(nrm, C.c_double), _p(other, C.c_int32))
        n = min(n, m)
        # corner: 0..7 box corner (on the plane, or inside box `other` >= 0), -1 ball on
        # the plane, -2 ball on box `body`
        return dict(body=body[:n], corner=corner[:n], x=x[:n], depth=d[:n], J=J[:n], normal=nrm[:n],
                    other=other[:n])

    def variant_state(self, vi: int):
        q, v, k, s = self.get_state()
        return (q[self.q_off[vi]:self.q_off[vi + 1]], v[self.v_off[vi]:self.v_off[vi + 1]], int(k[vi]), int(s[vi]))
