"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Bar: per-step relative state error <= 1e-4 (teacher
forced, outside the contact activation band) and fitness within 1e-3 relative
(floor 1 cm) after T steps, with a float32 sensitivity gate."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import workloads as W

from _parity import (FAIL_CAP, FIT_FLOOR, FIT_TOL, STEP_TOL, THREADS, FloatOracleSim, assert_gate, oracle_reference,
                     teacher_forced, teacher_forced_counters)

pytestmark = pytest.mark.gpu


def _sim(pop, **kw):
    from paper_2502_11129_amd.sim import Simulator
    return Simulator(pop, **kw)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name, pop, ks", [
    ("snake3 x16", W.snake(16), [0, 1, 5, 20, 60, 150, 300, 500, 750, 999]),
    ("boxes x128", W.boxes(128), [0, 1, 100, 200, 300, 450, 600, 1000, 1500, 1999]),
    ("trees spot-check x64", None, [0, 1, 10, 100, 400, 1000, 2000, 3000, 4999]),
    ("quadrupeds x16", W.quadrupeds(16), [0, 1, 10, 100, 300, 600, 999]),
    ("quadrupeds x16 long horizon", W.quadrupeds(16), [4999, 9999, 19999, 29999]),
    ("snake3 x16 started at (0.3, -0.2)", W.shifted(W.snake(16), 0.3, -0.2), [0, 1, 100, 500, 999]),
])
def test_teacher_forced_one_step(name, pop, ks):
    if pop is None:
        pop = W.random_trees(indices=W.TREE_SPOTCHECK)
    _say(f"[teacher-forced] {name}: {pop.n_variants} variants, steps {ks}")
    sim = _sim(pop)
    worst, in_band, errs = teacher_forced(pop, sim, ks)
    _say(f"  worst step error {worst:.3e} over {len(errs)} cases; {in_band} cases in the activation band")
    assert len(errs) > 0
    assert worst <= STEP_TOL


def _fitness_case(pop, T, **kw):
    sim = _sim(pop, **kw)
    sim.rollout(T)
    Fg = sim.fitness().astype(np.float64)
    Fr, F32, Fp, margin = oracle_reference(pop, T)
    return sim, Fg, Fr, F32, Fp, margin


# Share of a population allowed to miss its bar at 1e4 and 3e4 steps (all of
# them in a sensitive class), fixed before the GPU results: over that long,
# every quadruped's feet cross the plane thousands of times.
LONG_FAIL_CAP = 0.25


@pytest.mark.parametrize("name, make, T", [
    ("snake3 x16 T=1000", lambda: W.snake(16), 1000),
    ("snake3 x16 started at (0.3, -0.2) T=1000", lambda: W.shifted(W.snake(16), 0.3, -0.2), 1000),
    ("boxes x256 T=2000", lambda: W.boxes(256), 2000),
    ("trees spot-check x64 T=5000", lambda: W.random_trees(indices=W.TREE_SPOTCHECK), 5000),
    ("trees x24 started at (-1.5, 2.0) T=2000", lambda: W.shifted(W.random_trees(24), -1.5, 2.0), 2000),
    ("quadrupeds x32 T=1000", lambda: W.quadrupeds(32), 1000),
    ("quadrupeds x16 T=10000", lambda: W.quadrupeds(16), 10000),
])
def test_fitness_after_T(name, make, T):
    pop = make()
    _say(f"[fitness] {name}")
    sim, Fg, Fr, F32, Fp, margin = _fitness_case(pop, T)
    a, b, s = sim.counters()
    assert (s == 0).all()
    assert_gate(Fg, Fr, F32, Fp, say=_say, margin=margin, fail_cap=LONG_FAIL_CAP if T >= 10000 else FAIL_CAP)


def test_fitness_is_displacement_from_the_start():
    """A population moved away from the origin: every core's fitness is its
    displacement from its own start, the same as the unmoved population's up
    to rounding, and far from its distance to the origin.  A free-flying box
    started at (0.4, -0.7) has the closed form n dt |v_xy|."""
    pop = W.snake(16)
    T = 1000
    _say("[fitness] snake3 x16 at the origin and moved to (0.3, -0.2)")
    a = _sim(pop)
    a.rollout(T)
    b = _sim(W.shifted(pop, 0.3, -0.2))
    b.rollout(T)
    Fa, Fb = a.fitness().astype(np.float64), b.fitness().astype(np.float64)
    _say(f"  max |F_moved - F| {np.abs(Fb - Fa).max():.2e} m; fitness range {Fa.min():.3f} .. {Fa.max():.3f} m")
    assert (np.abs(Fb - Fa) <= FIT_TOL * np.maximum(Fa, FIT_FLOOR)).all()
    qb, _, _ = b.get_state()
    xy = np.stack([qb[pop.q_offset[:-1]], qb[pop.q_offset[:-1] + 1]], 1).astype(np.float64)
    assert (np.abs(np.linalg.norm(xy, axis=1) - Fb) > 1e-3).all()
    box = W.single_box(pos=(0.4, -0.7, 3.0), quat=(np.cos(0.35), 0.0, 0.0, np.sin(0.35)), v_b=(0.3, -0.2, 0.7))
    s = _sim(box)
    for n in (1, 37, 400):
        s.rollout(n)
        F = float(s.fitness()[0])
        exact = n * 0.002 * np.hypot(0.3, 0.2)
        assert abs(F - exact) <= FIT_TOL * max(exact, FIT_FLOOR), (n, F, exact)


def test_fitness_long_horizon():
    """30 000 steps (60 s) on 16 quadrupeds under the per-variant fitness
    gate, with the counts of variants within the bound, FP32-sensitive and
    relaxed printed; also the median relative deviation and the ranking of
    the variants (what selection uses), Spearman rho >= 0.95."""
    from scipy.stats import spearmanr
    pop = W.quadrupeds(16)
    T = 30000
    _say(f"[fitness, long horizon] quadrupeds x16 T={T}")
    sim, Fg, Fr, F32, Fp, margin = _fitness_case(pop, T)
    rel = np.abs(Fg - Fr) / np.maximum(np.abs(Fr), FIT_FLOOR)
    rho = spearmanr(Fg, Fr)[0]
    _say(f"  median rel dev {np.median(rel):.2e}, max {rel.max():.2e}, spearman {rho:.4f}")
    _, _, s = sim.counters()
    assert (s == 0).all() and np.isfinite(Fg).all()
    assert_gate(Fg, Fr, F32, Fp, say=_say, margin=margin, fail_cap=LONG_FAIL_CAP)
    assert np.median(rel) <= FIT_TOL
    assert rho >= 0.95


def test_teacher_forced_counters_exact():
    """The per-step counters (active contact rows, clamp rows engaged at the
    end of the step) of one GPU step from the oracle's state equal the
    oracle's exactly, for every case where the oracle's own float instance
    agrees with its FP64 counts (a case where even that disagrees sits on a
    contact or clamp switch, where single precision may flip the decision:
    counted and printed)."""
    for name, pop, ks in (("snake3 x16", W.snake(16), [0, 1, 50, 200, 500, 999]),
                          ("trees spot-check x64", W.random_trees(indices=W.TREE_SPOTCHECK),
                           [0, 1, 100, 400, 1000, 2500, 4999])):
        _say(f"[counters] {name}, steps {ks}")
        compared, skipped, nz = teacher_forced_counters(pop, _sim(pop), ks)
        _say(f"  {compared} (variant, step) cases equal ({nz} with contacts or clamps), {skipped} on a switch")
        assert compared > 0.9 * (compared + skipped) and nz > 0


def test_overflow_contacts_bitwise_equal_register_path():
    """Contacts beyond the register budget take the workspace path: same
    arithmetic, so results match the all-in-register kernel bit for bit."""
    pop = W.quadrupeds(9)          # 9: ragged last wave
    _say("[overflow] quadrupeds x9, contacts_in_registers 2 vs default, T=600")
    a = _sim(pop)
    b = _sim(pop, contacts_in_registers=2)
    a.rollout(600)
    b.rollout(600)
    qa, va, _ = a.get_state()
    qb, vb, _ = b.get_state()
    ca, _, _ = a.counters()
    assert ca.max() > 600 * 2      # the overflow path was exercised
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(va, vb)


def test_determinism_chunking_and_resume():
    pop = W.random_trees(37)
    _say("[determinism] trees x37")
    s1 = _sim(pop)
    s1.rollout(300)
    q1, v1, k1 = s1.get_state()
    s1.rollout(300)
    q2, v2, _ = s1.get_state()
    np.testing.assert_array_equal(q1, q2)
    np.testing.assert_array_equal(v1, v2)
    s2 = _sim(pop)
    for _ in range(3):
        s2.step(100)
    q3, v3, k3 = s2.get_state()
    np.testing.assert_array_equal(q1, q3)
    np.testing.assert_array_equal(k1, k3)
    # resume: stop at 150, reload the state into a fresh simulator, continue
    s3 = _sim(pop)
    s3.step(150)
    qm, vm, km = s3.get_state()
    s4 = _sim(pop)
    s4.set_state(qm, vm, km)
    s4.step(150)
    q4, v4, _ = s4.get_state()
    np.testing.assert_array_equal(q1, q4)
    np.testing.assert_array_equal(v1, v4)
    # step counter drives the CPG phase: the fitness reference is still k = 0
    F1 = s1.fitness()
    assert np.isfinite(F1).all()


def test_graph_replay_matches_eager():
    pop = W.snake(16)
    _say("[graph] snake3 x16, 4 replays")
    e = _sim(pop)
    e.rollout(400)
    Fe = e.fitness()
    g = _sim(pop, use_graph=True)
    for _ in range(4):
        g.rollout(400)
        np.testing.assert_array_equal(g.fitness(), Fe)
        e.step(3)                  # unrelated eager work between replays


def test_nonfinite_state_freezes_only_that_variant():
    pop = W.snake(8)
    _say("[failure] NaN injected into variant 3")
    a = _sim(pop)
    b = _sim(pop)
    q, v, k = a.get_state()
    v_bad = v.copy()
    v_bad[pop.v_offset[3] + 6] = np.nan
    b.set_state(q, v_bad, k)
    a.step(200)
    b.step(200)
    qa, va, _ = a.get_state()
    qb, vb, kb = b.get_state()
    _, _, s = b.counters()
    assert s[3] == 1 and (np.delete(s, 3) == 0).all()
    assert np.isnan(b.fitness()[3])
    keep = np.ones(len(qa), bool)
    keep[pop.q_offset[3]:pop.q_offset[4]] = False
    np.testing.assert_array_equal(qa[keep], qb[keep])
    assert kb[3] == 0 and kb[0] == 200


def test_fixed_root_pendulum_period_on_gpu():
    th_eq = np.pi / 2
    params = dict(W.DEFAULT_PARAMS, kp=0.0, kd=0.0)
    pop = W.chain(1, ["+x"], [W.AXIS_Y], root_type=W.ROOT_FIXED, root_pose=(0, 0, 1.0, 1, 0, 0, 0),
                  theta0=[th_eq + 0.01], params=params)
    _say("[closed form] compound pendulum on the GPU")
    sim = _sim(pop)
    n = 2050
    th = np.zeros(n)
    for i in range(n):
        sim.step(1)
        th[i] = sim.get_state()[0][0]
    x = th - th_eq
    up = np.where((x[:-1] < 0) & (x[1:] >= 0))[0]
    t_cross = (up + 1 - x[up + 1] / (x[up + 1] - x[up])) * 0.002
    T_exact = 2 * np.pi * np.sqrt(5.0 / 3.0 * 0.03 / 9.81)
    assert abs(np.diff(t_cross).mean() - T_exact) / T_exact < 1e-3


def test_free_fall_and_resting_box_on_gpu():
    _say("[closed form] free fall and resting cube on the GPU")
    pop = W.single_box(pos=(0.0, 0.0, 3.0), v_b=(0.3, -0.2, 0.7))
    sim = _sim(pop)
    sim.step(300)
    q, _, _ = sim.get_state()
    n, dt = 300, np.float32(0.002)
    z = np.float32(3.0) + n * dt * np.float32(0.7) - 9.81 * dt * dt * n * (n + 1) / 2
    assert abs(q[2] - z) < 2e-5
    cube = W.single_box(half=(0.05, 0.05, 0.05), pos=(0, 0, 0.05))
    sim = _sim(cube)
    sim.step(300)
    q, _, _ = sim.get_state()
    assert abs((0.05 - q[2]) - 9.81e-4) / 9.81e-4 < 0.05


def _star22():
    """22 hinges (nv = 28, the largest) as four limbs of 6, 6, 5, 5 bricks on
    the core faces, resting on the plane, with CPG drive."""
    parents, faces, axes = [], [], []
    for face, length in zip(W.CORE_SLOTS, (6, 6, 5, 5)):
        for j in range(length):
            parents.append(0 if j == 0 else len(parents))
            faces.append(face if j == 0 else "+x")
            axes.append(j % 2)
    rng = np.random.default_rng(99)
    cpg = np.stack([rng.uniform(0, 1, 22), rng.uniform(1, 6, 22), rng.uniform(0, 2 * np.pi, 22)], 1)
    return W.chain(22, faces, axes, root_type=W.ROOT_FREE, root_q=[0, 0, 0.05, 1, 0, 0, 0], parents=parents,
                   cpg=cpg, name="star22")


def test_edge_cases_sizes():
    """n = 1, n not a multiple of 4, nv = 28 (the largest), T = 0."""
    _say("[edge] single variant, ragged, nv=28, T=0")
    for pop in (W.snake(1), W.random_trees(5), _star22()):
        sim = _sim(pop)
        sim.rollout(0)
        assert (sim.fitness() == 0).all()
        sim.rollout(1000)
        Fg = sim.fitness().astype(np.float64)
        Fr, F32, Fp, margin = oracle_reference(pop, 1000)
        assert_gate(Fg, Fr, F32, Fp, say=_say, label=f"{pop.name}: ", margin=margin)


def _mt_condition(o, pop, q, v):
    """2-norm condition number of M~ = M + dt (kd + dt kp) S (the matrix every
    solve of the step uses) at a state, from the FP64 oracle's M."""
    M, _ = o.dynamics(0, q, v)
    p = pop.params
    r0 = 6 if pop.root_type == W.ROOT_FREE else 0
    Mt = M.copy()
    Mt[np.arange(r0, M.shape[0]), np.arange(r0, M.shape[0])] += p["dt"] * (p["kd"] + p["dt"] * p["kp"])
    return float(np.linalg.cond(Mt))


def test_ill_conditioned_chain_per_step_error():
    """20 bricks in a straight line (nv = 26, the largest tree of the spec)
    dropped flat: cond(M~) is about 1.9e4.  A float32 solve with M~ is accurate
    to about cond(M~) u (u = 2^-24) relative in the worst direction, 1.1e-3
    here, eleven times the 1e-4 bar: at the impact steps every float32
    computation of the step misses 1e-4 (the oracle's float instance, textbook
    Cholesky: 2.7e-4; the same with an explicit Gauss-Jordan inverse, with and
    without a refinement step: 1e-5 to 2.6e-4 from step to step).  Each step
    is therefore held to max(1e-4, cond(M~_k) u), the textbook forward-error
    bound of a backward-stable float32 solve, with cond(M~_k) from the FP64
    oracle's matrix at that step's state; the steps above 1e-4 are counted."""
    pop = W.chain(20, ["+x"] * 20, [0, 1] * 10, root_type=W.ROOT_FREE, root_q=[0, 0, 0.5, 1, 0, 0, 0])
    ks = [0, 1, 50, 100, 150, 151, 152, 153, 154, 155, 156, 158, 160, 165, 170, 180, 190, 199, 250, 300]
    _say(f"[teacher-forced] ill-conditioned chain nv=26, steps {ks}")
    worst, in_band, errs, where = teacher_forced(pop, _sim(pop), ks, keys=True)
    worst32, _, errs32, where32 = teacher_forced(pop, FloatOracleSim(pop), ks, keys=True)
    assert where == where32
    o = O.Oracle(pop)
    cond, cur = {}, 0
    for k in sorted(ks):
        o.step(k - cur, THREADS)
        cur = k
        q, v, _, _ = o.get_state()
        cond[k] = _mt_condition(o, pop, q, v)
    kappa = np.array([cond[w[0]] for w in where])
    bar = np.maximum(STEP_TOL, kappa * 2.0 ** -24)
    over = errs > STEP_TOL
    _say(f"  worst step error {worst:.3e} over {len(errs)} cases ({worst32:.3e} for the float oracle); "
         f"cond(M~) {kappa.min():.3g} .. {kappa.max():.3g}; {int(over.sum())} steps above 1e-4 "
         f"{[where[i][0] for i in np.where(over)[0]]} (float oracle: {int((errs32 > STEP_TOL).sum())}); "
         f"worst error / bar {np.max(errs / bar):.3f}; {in_band} cases in the activation band")
    assert len(errs) >= len(ks) - 3
    assert (errs <= bar).all(), [(where[i], errs[i], bar[i]) for i in np.where(errs > bar)[0]]


def test_split_rollout_gpu_part_bitwise_host_part_within_bar():
    """CPU/GPU split (paper Sec. 6): variants left on the GPU give bit-identical
    results to a GPU-only rollout; variants sent to host threads meet the
    oracle bar; the merged state is visible through the normal calls."""
    pop = W.random_trees(40)
    _say("[split] trees x40, 10 variants on host threads, T=400")
    g = _sim(pop)
    g.rollout(400)
    Fg = g.fitness()
    s = _sim(pop)
    t = s.rollout_split(400, n_host=10, threads=4)
    Fs = s.fitness()
    assert t["n_host"] == 10 and t["n_gpu"] == 30 and t["combined_s"] > 0
    Fr, F32, Fp, margin = oracle_reference(pop, 400)
    assert_gate(Fs.astype(np.float64), Fr, F32, Fp, say=_say, margin=margin)
    same = Fs == Fg
    assert same.sum() >= 30          # the GPU share is bit-identical
    _, _, k = s.get_state()
    assert (k == 400).all()


def test_split_rollout_requeues_a_failed_host_share_on_the_gpu():
    """Host workers that fail (forced from the host: the first three
    variants taken raise an error) drop out; the rest of the host share is
    finished by the other workers and the three are re-run on the GPU, so
    every variant has its result: re-queued and GPU-share variants bit for
    bit the GPU-only rollout's, host-finished ones within the oracle bar.
    With every worker failing, the whole host share is re-queued."""
    pop = W.random_trees(64)
    _say("[split re-queue] trees x64, 24 on 8 host threads, 3 forced failures, T=300")
    g = _sim(pop)
    g.rollout(300)
    Fg = g.fitness()
    qg, vg, kg = g.get_state()
    s = _sim(pop, host_fault_items=3)
    t = s.rollout_split(300, n_host=24, threads=8)
    assert t["n_requeued"] == 3 and t["n_host"] == 24
    Fs = s.fitness()
    assert np.isfinite(Fs).all()
    assert (Fs == Fg).sum() >= 40 + 3          # GPU share and re-queued variants
    Fr, F32, Fp, margin = oracle_reference(pop, 300)
    assert_gate(Fs.astype(np.float64), Fr, F32, Fp, say=_say, margin=margin)
    _, _, k = s.get_state()
    assert (k == 300).all()
    a = _sim(pop, host_fault_items=24)
    t = a.rollout_split(300, n_host=24, threads=1)
    assert t["n_requeued"] == 24
    q, v, k = a.get_state()
    np.testing.assert_array_equal(a.fitness(), Fg)
    np.testing.assert_array_equal(q, qg)
    np.testing.assert_array_equal(v, vg)
