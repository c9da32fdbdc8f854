"""GPU parity of the box-and-ball scene (a free ball per variant, ball-plane
and ball-box contacts): the ball kernels through the C ABI against the FP64
oracle, to the same bars as the plane-only scenes -- per-step relative state
error <= 1e-4 teacher forced (outside the contact activation band, which
here includes the ball's contact switches), and fitness within 1e-3 relative
after T steps with the float32 sensitivity gate."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import workloads as W

from _parity import STEP_TOL, THREADS, assert_gate, oracle_reference, teacher_forced, teacher_forced_counters

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _small_trees(n, key=1):
    """Random trees of at most 16 hinges (ball included, at most 28 DoFs)."""
    idx = [i for i in range(4 * n + 64) if len(W.random_tree(i)[0]) <= 16][:n]
    return W.attach_ball(W.random_trees(indices=idx), key=key)


CASES = {
    "box_and_ball": lambda: W.box_and_ball(64),
    "snake3+ball": lambda: W.attach_ball(W.snake(16)),
    "trees+ball": lambda: _small_trees(24),
}


@pytest.mark.parametrize("name, ks", [
    ("box_and_ball", [0, 1, 50, 150, 300, 450, 700, 1000, 1500]),
    ("snake3+ball", [0, 1, 20, 100, 250, 500, 900]),
    ("trees+ball", [0, 1, 20, 100, 300, 600]),
])
def test_ball_teacher_forced_one_step(name, ks):
    from paper_2502_11129_amd.sim import Simulator
    pop = CASES[name]()
    _say(f"[ball teacher-forced] {name}: {pop.n_variants} variants, steps {ks}")
    sim = Simulator(pop)
    worst, in_band, errs = teacher_forced(pop, sim, ks)
    _say(f"  worst step error {worst:.3e} over {len(errs)} cases; {in_band} in the activation band")
    assert len(errs) > 0
    assert worst <= STEP_TOL


@pytest.mark.parametrize("name, make, T", [
    ("box_and_ball x256 T=2000", lambda: W.box_and_ball(256), 2000),
    ("snake3+ball x16 T=1000", lambda: W.attach_ball(W.snake(16)), 1000),
    ("trees+ball x24 T=1000", lambda: _small_trees(24), 1000),
])
def test_ball_fitness_after_T(name, make, T):
    from paper_2502_11129_amd.sim import Simulator
    pop = make()
    _say(f"[ball fitness] {name}")
    sim = Simulator(pop)
    sim.rollout(T)
    Fg = sim.fitness().astype(np.float64)
    Fr, F32, Fp, margin = oracle_reference(pop, T)
    _, _, status = sim.counters()
    assert (status == 0).all()
    assert_gate(Fg, Fr, F32, Fp, say=_say, margin=margin)


def test_ball_overflow_contacts_bitwise_equal_register_path():
    """Ball contacts beyond the register budget take the workspace path with
    the same arithmetic: results equal the all-in-register run bit for bit."""
    from paper_2502_11129_amd.sim import Simulator
    pop = W.box_and_ball(9)                      # 9: ragged last wave
    _say("[ball overflow] box_and_ball x9, 2 contacts in registers vs 8, T=800")
    a = Simulator(pop)
    b = Simulator(pop, contacts_in_registers=2)
    assert [x[2] for x in a.bins()] == [8] and [x[2] for x in b.bins()] == [2]
    a.rollout(800)
    b.rollout(800)
    qa, va, _ = a.get_state()
    qb, vb, _ = b.get_state()
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(va, vb)
    np.testing.assert_array_equal(a.fitness(), b.fitness())


def test_ball_contact_row_counts_match_oracle():
    """Contact rows per step (box corners, ball-plane, ball-box) and engaged
    clamp rows of one GPU step from the oracle's state equal the oracle's
    exactly, wherever the oracle's float instance agrees with its FP64 counts."""
    from paper_2502_11129_amd.sim import Simulator
    for name, pop, ks in (("box_and_ball x32", W.box_and_ball(32), [0, 1, 50, 100, 200, 300, 600, 999]),
                          ("snake3+ball x16", W.attach_ball(W.snake(16)), [0, 1, 100, 300, 600, 999])):
        _say(f"[ball counters] {name}, steps {ks}")
        compared, skipped, nz = teacher_forced_counters(pop, Simulator(pop), ks)
        _say(f"  {compared} (variant, step) cases equal ({nz} with contacts or clamps), {skipped} on a switch")
        assert compared > 0.9 * (compared + skipped) and nz > 0
