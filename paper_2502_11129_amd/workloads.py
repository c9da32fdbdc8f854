"""Seeded synthetic populations of box-and-hinge robots.

This module only *draws inputs*: morphologies, CPG parameters and initial
states, as flat float32/int32 arrays in the variant-CSR layout that both the
HIP library and the FP64 checker accept.  It contains none of the simulation
arithmetic (no kinematics, dynamics, contact or integration); the one piece of
geometry here is the lift of a dropped box so that it starts above the ground,
which is part of drawing its initial state.

The paper (Sec. 4, "Simulation Parameters"; Sec. 6) benchmarks populations of
"variants" of MuJoCo scenes whose model files are not available.  The
populations below stand in for them; every draw uses
``numpy.random.default_rng([config, index])`` (PCG64 seeded through
SeedSequence) in a fixed order so that variant ``i`` of a config is the same
robot whatever the population size.

Conventions of the model layout (shared by every consumer):

* bodies of a variant are numbered in creation order, body 0 is the core
  (root), ``parent[b] < b``;
* each non-root body is joined to its parent by one hinge (DoF) located at
  the centre of a face of the parent (``anchor_parent``, parent frame); the
  child's rest orientation relative to the parent is ``rest_quat`` (w, x, y,
  z) and the child's back-face centre ``anchor_child`` sits on the anchor;
* the hinge axis ``axis`` is a unit vector in the child frame;
* ``cpg[b] = (A, omega, phi)`` drives the hinge of body ``b``;
* a FREE root has generalised position (p0, Q0, theta_1..theta_nh) and
  velocity (omega_body, v_body, thetadot_1..thetadot_nh); a FIXED root
  (used by unit tests only) has only the hinge coordinates and its pose is
  given by ``root_pose`` = (p0, Q0);
* optionally every variant of a population carries one free solid sphere
  (``ball`` = [radius, mass] per variant, the box-and-ball scene): its
  position (centre, Q) follows the robot's coordinates in q and its world
  angular velocity and centre velocity follow the robot's in v;
* ``self_collision`` adds contacts between the boxes of one robot that are
  not joined by a hinge.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import dataclasses

import numpy as np

ROOT_FREE = 0
ROOT_FIXED = 1

CORE_HALF = 0.05          # 0.1 m cube
CORE_MASS = 0.15
BRICK_HALF = 0.03         # 0.06 m cube
BRICK_MASS = 0.05
CORE_Z0 = 0.05            # core bottom face resting on the plane

# face name -> outward normal in the body frame
FACES = {
    "+x": (1.0, 0.0, 0.0), "-x": (-1.0, 0.0, 0.0),
    "+y": (0.0, 1.0, 0.0), "-y": (0.0, -1.0, 0.0),
    "+z": (0.0, 0.0, 1.0), "-z": (0.0, 0.0, -1.0),
}
CORE_SLOTS = ("+x", "-x", "+y", "-y")
BRICK_SLOTS = ("+x", "+y", "-y")
AXIS_Z = 0
AXIS_Y = 1

DEFAULT_PARAMS = dict(kp=5.0, kd=0.05, tau_max=0.9, k_contact=1.0e4,
                      b_contact=100.0, dt=0.002, gravity=(0.0, 0.0, -9.81),
                      pgs_iters=8)


def _face_rest_quat(face: str) -> tuple:
    """Rest rotation (w,x,y,z) taking the child's +x axis onto the face normal."""
    h = np.sqrt(0.5)
    return {
        "+x": (1.0, 0.0, 0.0, 0.0),
        "+y": (h, 0.0, 0.0, h),          # yaw +90 deg
        "-x": (0.0, 0.0, 0.0, 1.0),      # yaw 180 deg
        "-y": (h, 0.0, 0.0, -h),         # yaw -90 deg
        "+z": (h, 0.0, -h, 0.0),         # pitch -90 deg about y: +x -> +z
        "-z": (h, 0.0, h, 0.0),          # pitch +90 deg about y: +x -> -z
    }[face]


@dataclass
class Population:
    """A batch of variants in variant-CSR layout (host arrays)."""
    body_offset: np.ndarray          # int32 [N+1]
    parent: np.ndarray               # int32 [NB]  (variant-local, -1 for root)
    half_ext: np.ndarray             # float32 [NB,3]
    mass: np.ndarray                 # float32 [NB]
    anchor_parent: np.ndarray        # float32 [NB,3]
    anchor_child: np.ndarray         # float32 [NB,3]
    rest_quat: np.ndarray            # float32 [NB,4]
    axis: np.ndarray                 # float32 [NB,3]
    cpg: np.ndarray                  # float32 [NB,3]  (A, omega, phi); zero for root
    mu: np.ndarray                   # float32 [N]
    q0: np.ndarray                   # float32 CSR, nq per variant
    v0: np.ndarray                   # float32 CSR, nv per variant
    root_pose: np.ndarray            # float32 [N,7] (FIXED roots; zeros otherwise)
    root_type: int = ROOT_FREE
    params: dict = field(default_factory=lambda: dict(DEFAULT_PARAMS))
    name: str = ""
    steps: int = 0                   # horizon T of the workload
    lifted: int = 0                  # boxes lifted off the plane at creation
    ball: np.ndarray | None = None   # float32 [N,2] (radius, mass) of each variant's ball, or None
    self_collision: bool = False     # contacts between the boxes of one robot (not joined by a hinge)

    @property
    def n_variants(self) -> int:
        return int(self.body_offset.shape[0] - 1)

    @property
    def n_bodies(self) -> np.ndarray:
        return np.diff(self.body_offset).astype(np.int64)

    @property
    def n_hinges(self) -> np.ndarray:
        return self.n_bodies - 1

    @property
    def nq(self) -> np.ndarray:
        return self.n_hinges + (7 if self.root_type == ROOT_FREE else 0) + (7 if self.ball is not None else 0)

    @property
    def nv(self) -> np.ndarray:
        return self.n_hinges + (6 if self.root_type == ROOT_FREE else 0) + (6 if self.ball is not None else 0)

    @property
    def q_offset(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nq)]).astype(np.int64)

    @property
    def v_offset(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nv)]).astype(np.int64)

    def subset(self, idx) -> "Population":
        """Population made of the listed variants (in the given order)."""
        idx = np.asarray(idx, dtype=np.int64)
        bo, qo, vo = self.body_offset, self.q_offset, self.v_offset
        bsel = np.concatenate([np.arange(bo[i], bo[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
        qsel = np.concatenate([np.arange(qo[i], qo[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
        vsel = np.concatenate([np.arange(vo[i], vo[i + 1]) for i in idx]) if len(idx) else np.zeros(0, np.int64)
        nb = np.diff(bo)[idx]
        return Population(
            body_offset=np.concatenate([[0], np.cumsum(nb)]).astype(np.int32),
            parent=self.parent[bsel].copy(), half_ext=self.half_ext[bsel].copy(),
            mass=self.mass[bsel].copy(), anchor_parent=self.anchor_parent[bsel].copy(),
            anchor_child=self.anchor_child[bsel].copy(), rest_quat=self.rest_quat[bsel].copy(),
            axis=self.axis[bsel].copy(), cpg=self.cpg[bsel].copy(), mu=self.mu[idx].copy(),
            q0=self.q0[qsel].copy(), v0=self.v0[vsel].copy(),
            root_pose=self.root_pose[idx].copy(), root_type=self.root_type,
            params=dict(self.params), name=self.name, steps=self.steps,
            ball=None if self.ball is None else self.ball[idx].copy(), self_collision=self.self_collision)


class _Builder:
    """Accumulates robots body by body, then emits a Population."""

    def __init__(self, root_type=ROOT_FREE):
        self.root_type = root_type
        self.rows = dict(parent=[], half=[], mass=[], ap=[], ac=[], rq=[], axis=[], cpg=[])
        self.offsets = [0]
        self.mu, self.q0, self.v0, self.root_pose = [], [], [], []
        self.ball = []

    def add_body(self, parent, half, mass, face=None, parent_half=None, axis_flag=AXIS_Z,
                 cpg=(0.0, 0.0, 0.0)):
        r = self.rows
        r["parent"].append(parent)
        r["half"].append(tuple(half))
        r["mass"].append(mass)
        if parent < 0:
            r["ap"].append((0.0, 0.0, 0.0))
            r["ac"].append((0.0, 0.0, 0.0))
            r["rq"].append((1.0, 0.0, 0.0, 0.0))
            r["axis"].append((0.0, 0.0, 1.0))
        else:
            n = np.array(FACES[face])
            r["ap"].append(tuple(n * np.asarray(parent_half)))
            r["ac"].append((-half[0], 0.0, 0.0))
            r["rq"].append(_face_rest_quat(face))
            r["axis"].append((0.0, 0.0, 1.0) if axis_flag == AXIS_Z else (0.0, 1.0, 0.0))
        r["cpg"].append(tuple(cpg))

    def end_variant(self, mu, q0, v0, root_pose=(0, 0, 0, 1, 0, 0, 0), ball=None):
        self.ball.append(ball)
        self.offsets.append(len(self.rows["parent"]))
        self.mu.append(mu)
        self.q0.extend(q0)
        self.v0.extend(v0)
        self.root_pose.append(tuple(root_pose))

    def build(self, name, steps, params=None, lifted=0) -> Population:
        r = self.rows
        f32 = lambda x, s: np.asarray(x, dtype=np.float32).reshape(s)
        nbt = len(r["parent"])
        return Population(
            body_offset=np.asarray(self.offsets, dtype=np.int32),
            parent=np.asarray(r["parent"], dtype=np.int32),
            half_ext=f32(r["half"], (nbt, 3)), mass=f32(r["mass"], (nbt,)),
            anchor_parent=f32(r["ap"], (nbt, 3)), anchor_child=f32(r["ac"], (nbt, 3)),
            rest_quat=f32(r["rq"], (nbt, 4)), axis=f32(r["axis"], (nbt, 3)),
            cpg=f32(r["cpg"], (nbt, 3)), mu=f32(self.mu, (-1,)),
            q0=f32(self.q0, (-1,)), v0=f32(self.v0, (-1,)),
            root_pose=f32(self.root_pose, (-1, 7)), root_type=self.root_type,
            params=dict(DEFAULT_PARAMS if params is None else params),
            name=name, steps=steps, lifted=lifted, ball=self._balls())

    def _balls(self):
        has = [bl is not None for bl in self.ball]
        if any(has) and not all(has):
            raise ValueError("either every variant has a ball or none does")
        return np.asarray(self.ball, dtype=np.float32).reshape(-1, 2) if has and all(has) else None


def _robot_state(nh):
    """Initial state of a legged robot: core on the plane, all hinges at 0, at rest."""
    q0 = [0.0, 0.0, CORE_Z0, 1.0, 0.0, 0.0, 0.0] + [0.0] * nh
    v0 = [0.0] * (6 + nh)
    return q0, v0


def _cpg_draw(rng, n):
    A = rng.uniform(0.0, 1.0, n)
    om = rng.uniform(1.0, 6.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    return A, om, ph


# ----------------------------------------------------------------------------
# Config C0: plain method -- 3-hinge snake
# ----------------------------------------------------------------------------
def snake(n=16, first=0):
    """16 snakes: core + 3 bricks chained on +x faces, axes z, y, z."""
    b = _Builder()
    axes = (AXIS_Z, AXIS_Y, AXIS_Z)
    for i in range(first, first + n):
        rng = np.random.default_rng([0, i])
        A, om, ph = _cpg_draw(rng, 3)
        b.add_body(-1, (CORE_HALF,) * 3, CORE_MASS)
        for j in range(3):
            ph_half = (CORE_HALF,) * 3 if j == 0 else (BRICK_HALF,) * 3
            b.add_body(j, (BRICK_HALF,) * 3, BRICK_MASS, "+x", ph_half, axes[j],
                       (A[j], om[j], ph[j]))
        q0, v0 = _robot_state(3)
        b.end_variant(1.0, q0, v0)
    return b.build("snake3", 1000)


# ----------------------------------------------------------------------------
# Config C1: box environment -- free boxes dropped on a plane
# ----------------------------------------------------------------------------
def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def boxes(n=4096, first=0, clearance=0.005):
    """Free boxes: sides U(0.05,0.3), density 1000, centre height U(0.2,1.0),
    uniform random orientation, world velocities N(0, 0.5), mu U(0.3, 1.2).

    A box whose lowest corner would start below ``clearance`` is raised so that
    it starts there (the count is kept in ``Population.lifted``)."""
    b = _Builder()
    lifted = 0
    for i in range(first, first + n):
        rng = np.random.default_rng([1, i])
        sides = rng.uniform(0.05, 0.3, 3)
        H = rng.uniform(0.2, 1.0)
        q = rng.normal(0.0, 1.0, 4)
        q /= np.linalg.norm(q)
        if q[0] < 0:
            q = -q
        vw = rng.normal(0.0, 0.5, 3)
        ww = rng.normal(0.0, 0.5, 3)
        mu = rng.uniform(0.3, 1.2)
        half = sides / 2.0
        R = _quat_to_rot(q)
        lowest = H - np.abs(R[2]) @ half
        if lowest < clearance:
            H += clearance - lowest
            lifted += 1
        m = 1000.0 * sides.prod()
        b.add_body(-1, tuple(half), m)
        vb = R.T @ vw
        wb = R.T @ ww
        b.end_variant(mu, [0.0, 0.0, H, *q], [*wb, *vb])
    return b.build("boxes", 2000, lifted=lifted)


# ----------------------------------------------------------------------------
# Config C2: uneven modular robots -- random trees of 4..20 hinges
# ----------------------------------------------------------------------------
MAX_DEPTH = 4


def random_tree(i):
    """Topology of variant i of the random-tree config: list of
    (parent, face, axis_flag) per brick, plus CPG draws."""
    rng = np.random.default_rng([2, i])
    nh = int(rng.integers(4, 21))
    depth = [0]
    used = [set()]
    bricks = []
    for _ in range(nh):
        free = []
        for body in range(len(depth)):
            if depth[body] >= MAX_DEPTH:
                continue
            for f in (CORE_SLOTS if body == 0 else BRICK_SLOTS):
                if f not in used[body]:
                    free.append((body, f))
        body, f = free[int(rng.integers(len(free)))]
        flag = int(rng.integers(2))
        used[body].add(f)
        used.append(set())
        depth.append(depth[body] + 1)
        bricks.append((body, f, flag))
    A, om, ph = _cpg_draw(rng, nh)
    return bricks, A, om, ph


def random_trees(n=8192, first=0, indices=None):
    b = _Builder()
    idx = range(first, first + n) if indices is None else indices
    for i in idx:
        bricks, A, om, ph = random_tree(int(i))
        b.add_body(-1, (CORE_HALF,) * 3, CORE_MASS)
        for j, (par, f, flag) in enumerate(bricks):
            ph_half = (CORE_HALF,) * 3 if par == 0 else (BRICK_HALF,) * 3
            b.add_body(par, (BRICK_HALF,) * 3, BRICK_MASS, f, ph_half, flag, (A[j], om[j], ph[j]))
        q0, v0 = _robot_state(len(bricks))
        b.end_variant(1.0, q0, v0)
    return b.build("trees", 5000)


# ----------------------------------------------------------------------------
# Config C3: long-horizon quadrupeds -- core + four 5-brick limbs
# ----------------------------------------------------------------------------
def quadrupeds(n=32768, first=0, steps=1000):
    b = _Builder()
    axes = (AXIS_Z, AXIS_Y, AXIS_Z, AXIS_Y, AXIS_Z)
    for i in range(first, first + n):
        rng = np.random.default_rng([3, i])
        A, om, ph = _cpg_draw(rng, 20)
        b.add_body(-1, (CORE_HALF,) * 3, CORE_MASS)
        for limb, face in enumerate(CORE_SLOTS):
            for j in range(5):
                h = limb * 5 + j
                if j == 0:
                    b.add_body(0, (BRICK_HALF,) * 3, BRICK_MASS, face, (CORE_HALF,) * 3, axes[j],
                               (A[h], om[h], ph[h]))
                else:
                    b.add_body(limb * 5 + j, (BRICK_HALF,) * 3, BRICK_MASS, "+x", (BRICK_HALF,) * 3,
                               axes[j], (A[h], om[h], ph[h]))
        q0, v0 = _robot_state(20)
        b.end_variant(1.0, q0, v0)
    return b.build("quadrupeds", steps)


# ----------------------------------------------------------------------------
# Small hand-built models used by unit tests
# ----------------------------------------------------------------------------
def chain(n_hinges, faces, axis_flags, root_type=ROOT_FIXED, root_pose=(0, 0, 1.0, 1, 0, 0, 0),
          theta0=None, thetadot0=None, root_q=None, root_v=None, parents=None, cpg=None,
          mu=1.0, params=None, name="chain"):
    """One variant: core plus ``n_hinges`` bricks.  ``parents`` defaults to a
    chain; ``faces`` and ``axis_flags`` give each brick's parent face and axis."""
    b = _Builder(root_type)
    parents = list(range(n_hinges)) if parents is None else list(parents)
    b.add_body(-1, (CORE_HALF,) * 3, CORE_MASS)
    for j in range(n_hinges):
        par = parents[j]
        ph_half = (CORE_HALF,) * 3 if par == 0 else (BRICK_HALF,) * 3
        c = (0.0, 0.0, 0.0) if cpg is None else tuple(cpg[j])
        b.add_body(par, (BRICK_HALF,) * 3, BRICK_MASS, faces[j], ph_half, axis_flags[j], c)
    th = [0.0] * n_hinges if theta0 is None else list(theta0)
    thd = [0.0] * n_hinges if thetadot0 is None else list(thetadot0)
    if root_type == ROOT_FREE:
        rq = [0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0] if root_q is None else list(root_q)
        rv = [0.0] * 6 if root_v is None else list(root_v)
        b.end_variant(mu, rq + th, rv + thd)
    else:
        b.end_variant(mu, th, thd, root_pose)
    return b.build(name, 0, params=params)


def nudged(pop: Population, seed: int) -> Population:
    """The population with every initial position coordinate moved by one
    float32 ulp, up or down by a draw of rng([7, seed]): two rollouts from pop
    and from nudged(pop) are equally correct float32 simulations of the same
    robots, so how far their rankings agree bounds what any predictor of the
    simulated fitness can reach."""
    rng = np.random.default_rng([7, seed])
    q0 = np.asarray(pop.q0, np.float32)
    up = rng.uniform(size=q0.shape) < 0.5
    q0 = np.where(up, np.nextafter(q0, np.float32(np.inf)), np.nextafter(q0, np.float32(-np.inf))).astype(np.float32)
    return dataclasses.replace(pop, q0=q0)


def twisted_chains(n=16, nh=6, root_type=ROOT_FREE, key=13):
    """Self-collision scene whose bricks cross edge to edge: n chains of nh
    bricks, each on a face drawn from +x / +y / -y of its parent with a drawn
    axis flag, driven by CPG parameters A ~ U(0.7, 1), omega ~ U(1.5, 4),
    phi ~ U(0, 2 pi) from rng([key, i, attempt]) (large amplitudes curl the
    chains into themselves); a FREE root rests on the plane, a FIXED one hangs
    at 1 m.  A draw whose rest pose (all angles 0: the chain turns left on
    +y, right on -y, in the plane) puts two boxes into each other is drawn
    again (attempt + 1)."""
    def overlapping(faces):
        pos, head, half = [(0.0, 0.0)], 0, [CORE_HALF]
        for f in faces:
            head = (head + {"+x": 0, "+y": 1, "-y": 3}[f]) % 4
            dx, dy = [(1, 0), (0, 1), (-1, 0), (0, -1)][head]
            r = half[-1] + BRICK_HALF
            pos.append((pos[-1][0] + r * dx, pos[-1][1] + r * dy))
            half.append(BRICK_HALF)
        for a in range(len(pos)):
            for b in range(a + 2, len(pos)):
                lim = half[a] + half[b] - 1e-9
                if abs(pos[a][0] - pos[b][0]) < lim and abs(pos[a][1] - pos[b][1]) < lim:
                    return True
        return False

    pops = []
    for i in range(n):
        for attempt in range(1000):
            rng = np.random.default_rng([key, i, attempt])
            flags = [int(x) for x in rng.integers(0, 2, nh)]
            faces = [str(x) for x in rng.choice(["+x", "+y", "-y"], nh)]
            if not overlapping(faces):
                break
        cpg = [(float(rng.uniform(0.7, 1.0)), float(rng.uniform(1.5, 4.0)), float(rng.uniform(0, 2 * np.pi)))
               for _ in range(nh)]
        if root_type == ROOT_FREE:
            pops.append(chain(nh, faces, flags, root_type=ROOT_FREE, root_q=[0, 0, CORE_HALF, 1, 0, 0, 0], cpg=cpg,
                              name="twisted chains"))
        else:
            pops.append(chain(nh, faces, flags, root_type=ROOT_FIXED, cpg=cpg, name="twisted chains"))
    return dataclasses.replace(concat(pops), self_collision=True, name="twisted chains")


def tilted(pop: Population, seed: int, angle=0.12) -> Population:
    """The population with every brick's rest orientation turned by a random
    rotation of at most ``angle`` rad about each axis (rotation vector drawn
    from U(-angle, angle)^3 with rng(seed)), composed on the right: hinge axes
    and box faces of different bricks are no longer exactly parallel or
    coplanar, so box pairs rarely sit exactly on a contact switch."""
    rng = np.random.default_rng(seed)
    rq = pop.rest_quat.astype(np.float64).copy()
    for b in range(len(rq)):
        if pop.parent[b] < 0:
            continue
        w = rng.uniform(-angle, angle, 3)
        th = float(np.linalg.norm(w))
        k = w / th
        d = np.concatenate([[np.cos(th / 2)], np.sin(th / 2) * k])
        a = rq[b]
        rq[b] = [a[0] * d[0] - a[1] * d[1] - a[2] * d[2] - a[3] * d[3],
                 a[0] * d[1] + a[1] * d[0] + a[2] * d[3] - a[3] * d[2],
                 a[0] * d[2] - a[1] * d[3] + a[2] * d[0] + a[3] * d[1],
                 a[0] * d[3] + a[1] * d[2] - a[2] * d[1] + a[3] * d[0]]
    return dataclasses.replace(pop, rest_quat=rq.astype(pop.rest_quat.dtype))


def single_box(half=(0.05, 0.05, 0.05), mass=None, pos=(0, 0, 1.0), quat=(1, 0, 0, 0),
               omega_b=(0, 0, 0), v_b=(0, 0, 0), mu=1.0, params=None, name="box", ball=None):
    """One free box; ``ball`` = dict(r, m, pos, quat, w, v) adds a ball
    (world angular velocity w and centre velocity v)."""
    b = _Builder()
    m = 1000.0 * 8 * np.prod(half) if mass is None else mass
    b.add_body(-1, tuple(half), m)
    q0, v0, bl = [*pos, *quat], [*omega_b, *v_b], None
    if ball is not None:
        q0 += [*ball["pos"], *ball.get("quat", (1.0, 0.0, 0.0, 0.0))]
        v0 += [*ball.get("w", (0.0, 0.0, 0.0)), *ball.get("v", (0.0, 0.0, 0.0))]
        bl = (ball["r"], ball["m"])
    b.end_variant(mu, q0, v0, ball=bl)
    return b.build(name, 0, params=params)


def concat(pops) -> Population:
    """Concatenate populations that share root type and parameters (and
    either all carry a ball or none does)."""
    p0 = pops[0]
    has_ball = [p.ball is not None for p in pops]
    if any(has_ball) and not all(has_ball):
        raise ValueError("cannot mix populations with and without a ball")
    if len(set(bool(p.self_collision) for p in pops)) > 1:
        raise ValueError("cannot mix populations with and without self-collision")
    nb = np.concatenate([p.n_bodies for p in pops])
    cat = lambda a: np.concatenate([getattr(p, a) for p in pops])
    return Population(
        body_offset=np.concatenate([[0], np.cumsum(nb)]).astype(np.int32),
        parent=cat("parent"), half_ext=cat("half_ext"), mass=cat("mass"),
        anchor_parent=cat("anchor_parent"), anchor_child=cat("anchor_child"),
        rest_quat=cat("rest_quat"), axis=cat("axis"), cpg=cat("cpg"), mu=cat("mu"),
        q0=cat("q0"), v0=cat("v0"), root_pose=cat("root_pose"), root_type=p0.root_type,
        params=dict(p0.params), name="+".join(p.name for p in pops), steps=p0.steps,
        ball=cat("ball") if all(has_ball) else None, self_collision=p0.self_collision)


def shifted(pop: Population, dx: float, dy: float) -> Population:
    """The same population with every free core (and ball) started
    (dx, dy) away in the horizontal plane: a rigid translation of the scene,
    which leaves every trajectory's displacement unchanged."""
    if pop.root_type != ROOT_FREE:
        raise ValueError("shifted() moves free cores; fixed roots carry their pose in root_pose")
    q0 = pop.q0.copy()
    qo = pop.q_offset
    for i in range(pop.n_variants):
        q0[qo[i]] += np.float32(dx)
        q0[qo[i] + 1] += np.float32(dy)
        if pop.ball is not None:
            q0[qo[i + 1] - 7] += np.float32(dx)
            q0[qo[i + 1] - 6] += np.float32(dy)
    return dataclasses.replace(pop, q0=q0, name=f"{pop.name}@({dx:g},{dy:g})")


# ----------------------------------------------------------------------------
# Box-and-ball scene: a free box and a free ball dropped on the plane
# ----------------------------------------------------------------------------
BALL_DENSITY = 1000.0


def _ball_mass(r, density=BALL_DENSITY):
    return density * 4.0 / 3.0 * np.pi * r ** 3


def box_and_ball(n=131072, first=0, clearance=0.005, steps=1000):
    """Box-and-ball variants: the box of ``boxes`` (sides U(0.05,0.3), density
    1000, uniform orientation, centre height U(0.2,1.0), world velocities
    N(0,0.5), mu U(0.3,1.2)) and a ball of radius U(0.03,0.15), density 1000,
    dropped from 0.05-0.5 m above the box top at a horizontal offset N(0,0.02)
    from the box centre, moving with the box (world velocity the box's plus
    N(0,0.1)) so that most balls land on it, angular velocity N(0,2)."""
    b = _Builder()
    lifted = 0
    for i in range(first, first + n):
        rng = np.random.default_rng([7, i])
        sides = rng.uniform(0.05, 0.3, 3)
        H = rng.uniform(0.2, 1.0)
        q = rng.normal(0.0, 1.0, 4)
        q /= np.linalg.norm(q)
        if q[0] < 0:
            q = -q
        vw = rng.normal(0.0, 0.5, 3)
        ww = rng.normal(0.0, 0.5, 3)
        mu = rng.uniform(0.3, 1.2)
        r = rng.uniform(0.03, 0.15)
        off = rng.normal(0.0, 0.02, 2)
        gap = rng.uniform(0.05, 0.5)
        bv = vw + rng.normal(0.0, 0.1, 3)
        bw = rng.normal(0.0, 2.0, 3)
        half = sides / 2.0
        R = _quat_to_rot(q)
        reach = np.abs(R[2]) @ half
        if H - reach < clearance:
            H += clearance - (H - reach)
            lifted += 1
        m = 1000.0 * sides.prod()
        b.add_body(-1, tuple(half), m)
        zb = H + reach + gap + r
        b.end_variant(mu, [0.0, 0.0, H, *q, off[0], off[1], zb, 1.0, 0.0, 0.0, 0.0],
                      [*(R.T @ ww), *(R.T @ vw), *bw, *bv], ball=(r, _ball_mass(r)))
    return b.build("box_and_ball", steps, lifted=lifted)


def attach_ball(pop: Population, key=0, radius=(0.03, 0.08), speed=(0.0, 1.0)) -> Population:
    """The same robots, each with a ball resting on the plane 0.15-0.35 m
    from its core in a random direction and rolling towards it (radius
    U(radius), density U(200,1000), speed U(speed)).  FREE roots only."""
    if pop.root_type != ROOT_FREE or pop.ball is not None:
        raise ValueError("attach_ball needs FREE roots without a ball")
    n = pop.n_variants
    qo, vo = pop.q_offset, pop.v_offset
    q0, v0, ball = [], [], np.zeros((n, 2), np.float32)
    for i in range(n):
        rng = np.random.default_rng([8, key, i])
        r = rng.uniform(*radius)
        rho = rng.uniform(200.0, 1000.0)
        dist = rng.uniform(0.15, 0.35)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        sp = rng.uniform(*speed)
        qi = pop.q0[qo[i]:qo[i + 1]]
        c = np.array([qi[0] + dist * np.cos(ang), qi[1] + dist * np.sin(ang), r + 1e-3])
        u = -np.array([np.cos(ang), np.sin(ang), 0.0])
        q0.append(np.concatenate([qi, c, [1.0, 0.0, 0.0, 0.0]]))
        v0.append(np.concatenate([pop.v0[vo[i]:vo[i + 1]], [0.0, 0.0, 0.0], sp * u]))
        ball[i] = (r, _ball_mass(r, rho))
    out = pop.subset(np.arange(n))
    out.q0 = np.concatenate(q0).astype(np.float32)
    out.v0 = np.concatenate(v0).astype(np.float32)
    out.ball = ball
    out.name = pop.name + "+ball"
    return out


CONFIGS = {
    "snake3": snake,
    "boxes": boxes,
    "trees": random_trees,
    "quadrupeds": quadrupeds,
    "box_and_ball": box_and_ball,
}

# Oracle spot-check subset of the random-tree population: indices 128*m.
TREE_SPOTCHECK = tuple(128 * m for m in range(64))


# ----------------------------------------------------------------------------
# Genotypes of random-tree robots (inputs of the learned surrogate)
# ----------------------------------------------------------------------------
FACE_CODE = {"+x": 0, "-x": 1, "+y": 2, "-y": 3}
FACE_NAME = ("+x", "-x", "+y", "-y")


@dataclass
class Genotypes:
    """Random-tree robots in compact form: hinge j joins body j+1 to
    parent[j] on face face[j] (0 +x, 1 -x, 2 +y, 3 -y in the parent frame)
    with axis flag axis[j] (0 child z, 1 child y); cpg[j] = (A, omega, phi).
    Padding: parent = face = axis = -1, cpg = 0."""
    nh: np.ndarray       # int32 [N]
    parent: np.ndarray   # int32 [N, 20]
    face: np.ndarray     # int32 [N, 20]
    axis: np.ndarray     # int32 [N, 20]
    cpg: np.ndarray      # float32 [N, 20, 3]

    def __len__(self):
        return int(self.nh.shape[0])

    def take(self, idx):
        idx = np.asarray(idx)
        return Genotypes(self.nh[idx], self.parent[idx], self.face[idx], self.axis[idx], self.cpg[idx])


def _empty_genotypes(n):
    return Genotypes(np.zeros(n, np.int32), -np.ones((n, 20), np.int32), -np.ones((n, 20), np.int32),
                     -np.ones((n, 20), np.int32), np.zeros((n, 20, 3), np.float32))


def tree_genotypes(indices) -> Genotypes:
    """Genotypes of the random-tree population (same robots as random_trees)."""
    indices = list(indices)
    g = _empty_genotypes(len(indices))
    for r, i in enumerate(indices):
        bricks, A, om, ph = random_tree(int(i))
        nh = len(bricks)
        g.nh[r] = nh
        for j, (par, f, flag) in enumerate(bricks):
            g.parent[r, j] = par
            g.face[r, j] = FACE_CODE[f]
            g.axis[r, j] = flag
        g.cpg[r, :nh, 0] = A
        g.cpg[r, :nh, 1] = om
        g.cpg[r, :nh, 2] = ph
    return g


def random_genotypes(n, key=0, chunk=262144) -> Genotypes:
    """n candidates drawn from the random-tree distribution (4..20 hinges,
    free-slot attachment on bodies of depth < 4, axis z/y, CPG ranges as for
    the snake), vectorised over candidates; seeded by rng([4, key, chunk])."""
    out = _empty_genotypes(n)
    # slot codes per body: core uses faces 0..3, bricks use +x, +y, -y (0, 2, 3)
    allowed = np.ones((21, 4), bool)
    allowed[1:, 1] = False
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        rng = np.random.default_rng([4, key, c0 // chunk])
        nh = rng.integers(4, 21, m)
        used = np.zeros((m, 21, 4), bool)
        depth = np.zeros((m, 21), np.int64)
        par = -np.ones((m, 20), np.int64)
        face = -np.ones((m, 20), np.int64)
        flag = -np.ones((m, 20), np.int64)
        u = rng.random((m, 20))
        fl = rng.integers(0, 2, (m, 20))
        rows = np.arange(m)
        for j in range(20):
            act = nh > j
            nbod = j + 1                                   # bodies existing before hinge j
            free = (~used[:, :nbod, :]) & allowed[None, :nbod, :] & (depth[:, :nbod, None] < 4)
            free = free.reshape(m, -1)
            cnt = free.sum(axis=1)
            pick = np.minimum((u[:, j] * cnt).astype(np.int64), np.maximum(cnt - 1, 0))
            csum = np.cumsum(free, axis=1)
            slot = np.argmax(csum > pick[:, None], axis=1)
            b, f = slot // 4, slot % 4
            a = act & (cnt > 0)
            used[rows[a], b[a], f[a]] = True
            depth[rows[a], j + 1] = depth[rows[a], b[a]] + 1
            par[a, j], face[a, j], flag[a, j] = b[a], f[a], fl[a, j]
        A = rng.uniform(0.0, 1.0, (m, 20))
        om = rng.uniform(1.0, 6.0, (m, 20))
        ph = rng.uniform(0.0, 2.0 * np.pi, (m, 20))
        pad = np.arange(20)[None, :] >= nh[:, None]
        sl = slice(c0, c0 + m)
        out.nh[sl] = nh
        out.parent[sl] = par
        out.face[sl] = face
        out.axis[sl] = flag
        cpg = np.stack([A, om, ph], axis=-1)
        cpg[pad] = 0.0
        out.cpg[sl] = cpg.astype(np.float32)
    return out


_FACE_VEC = np.array([FACES[f] for f in FACE_NAME], np.float32)                  # [4, 3]
_FACE_QUAT = np.array([_face_rest_quat(f) for f in FACE_NAME], np.float32)        # [4, 4]


def population_from_genotypes(g: Genotypes, steps=5000) -> Population:
    """Robots of the given genotypes (core + bricks, as in random_trees),
    assembled with array operations; the same arrays as building them body
    by body (``_population_from_genotypes_bodywise``)."""
    n = len(g)
    nh = np.asarray(g.nh, np.int64)
    nb = nh + 1
    bo = np.concatenate([[0], np.cumsum(nb)]).astype(np.int32)
    NB = int(bo[-1])
    var = np.repeat(np.arange(n), nb)                       # variant of each body
    loc = np.arange(NB) - np.repeat(bo[:-1], nb)            # body index within its variant
    core = loc == 0
    j = np.where(core, 0, loc - 1)                          # hinge of a brick
    par = np.where(core, -1, g.parent[var, j]).astype(np.int32)
    fcode = np.where(core, 0, g.face[var, j]).astype(np.int64)
    flag = np.where(core, 0, g.axis[var, j])
    half = np.where(core[:, None], np.float32(CORE_HALF), np.float32(BRICK_HALF)).repeat(3, axis=1).astype(np.float32)
    mass = np.where(core, np.float32(CORE_MASS), np.float32(BRICK_MASS)).astype(np.float32)
    parent_half = np.where(par == 0, CORE_HALF, BRICK_HALF)
    ap = np.where(core[:, None], 0.0, _FACE_VEC[fcode].astype(np.float64) * parent_half[:, None]).astype(np.float32)
    ac = np.zeros((NB, 3), np.float32)
    ac[~core, 0] = -BRICK_HALF
    rq = np.where(core[:, None], np.array([1, 0, 0, 0], np.float32), _FACE_QUAT[fcode]).astype(np.float32)
    axis = np.where((flag == 0)[:, None], np.array([0, 0, 1], np.float32), np.array([0, 1, 0], np.float32))
    axis = axis.astype(np.float32)
    cpg = np.where(core[:, None], 0.0, g.cpg[var, j]).astype(np.float32)
    nq = 7 + nh
    q0 = np.zeros(int(nq.sum()), np.float32)
    qo = np.concatenate([[0], np.cumsum(nq)])[:-1]
    q0[qo + 2] = CORE_Z0
    q0[qo + 3] = 1.0
    v0 = np.zeros(int((6 + nh).sum()), np.float32)
    root_pose = np.tile(np.array([0, 0, 0, 1, 0, 0, 0], np.float32), (n, 1))
    return Population(body_offset=bo, parent=par, half_ext=half, mass=mass, anchor_parent=ap, anchor_child=ac,
                      rest_quat=rq, axis=axis, cpg=cpg, mu=np.ones(n, np.float32), q0=q0, v0=v0,
                      root_pose=root_pose, root_type=ROOT_FREE, params=dict(DEFAULT_PARAMS), name="genotypes",
                      steps=steps)


def _population_from_genotypes_bodywise(g: Genotypes, steps=5000) -> Population:
    """Robots of the given genotypes built body by body (reference for the
    array version above)."""
    b = _Builder()
    for i in range(len(g)):
        nh = int(g.nh[i])
        b.add_body(-1, (CORE_HALF,) * 3, CORE_MASS)
        for j in range(nh):
            par = int(g.parent[i, j])
            ph_half = (CORE_HALF,) * 3 if par == 0 else (BRICK_HALF,) * 3
            b.add_body(par, (BRICK_HALF,) * 3, BRICK_MASS, FACE_NAME[int(g.face[i, j])], ph_half,
                       int(g.axis[i, j]), tuple(float(x) for x in g.cpg[i, j]))
        q0, v0 = _robot_state(nh)
        b.end_variant(1.0, q0, v0)
    return b.build("genotypes", steps)


# ----------------------------------------------------------------------------
# Initial parameters of the surrogate network (drawn here, passed in)
# ----------------------------------------------------------------------------
MLP_DIMS = (128, 256, 256, 256, 1)


def mlp_init(seed=0) -> np.ndarray:
    """Flat float32 parameters (W1, b1, W2, b2, W3, b3, W4, b4; W_l[in][out]
    row-major), every entry U(-1/sqrt(fan_in), +1/sqrt(fan_in)); seeded by
    rng([5, seed])."""
    rng = np.random.default_rng([5, seed])
    parts = []
    for l in range(4):
        lim = 1.0 / np.sqrt(MLP_DIMS[l])
        parts.append(rng.uniform(-lim, lim, MLP_DIMS[l] * MLP_DIMS[l + 1]))
        parts.append(rng.uniform(-lim, lim, MLP_DIMS[l + 1]))
    return np.concatenate(parts).astype(np.float32)


def genotype_arrays(g: Genotypes) -> dict:
    """The genotype arrays in the element types the surrogate library reads."""
    return dict(nh=np.ascontiguousarray(g.nh, np.int32), parent=np.ascontiguousarray(g.parent, np.int8),
                face=np.ascontiguousarray(g.face, np.int8), axis=np.ascontiguousarray(g.axis, np.int8),
                cpg=np.ascontiguousarray(g.cpg, np.float32))
