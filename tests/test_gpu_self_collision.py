"""GPU parity of self-collision (corners of a box inside another box of the
same robot, one separating-axis normal per pair; one contact where two
edges cross with no corner inside): the self-collision kernels
through the C ABI against the FP64 oracle, to the bars of the other scenes --
per-step relative state error <= 1e-4 teacher forced (outside the activation
band, widened to the self-contact switches: a corner near another box's
surface, near-ties of the separating axis), fitness within 1e-3 relative
after T with the float32 sensitivity gate, and the overflow path bitwise
equal to the in-register one."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import workloads as W

from _parity import STEP_TOL, THREADS, FloatOracleSim, assert_gate, oracle_reference, teacher_forced

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _self(pop):
    return dataclasses.replace(pop, self_collision=True)


def _folding_chains():
    """FIXED-root 4-brick chains driven to curl onto their core."""
    pops = []
    for i in range(6):
        rng = np.random.default_rng([11, i])
        cpg = [(float(rng.uniform(0.8, 1.0)), float(rng.uniform(1.5, 3.0)), float(rng.uniform(0, 6.28)))] * 4
        pops.append(W.chain(4, ["+x"] * 4, [0] * 4, root_type=W.ROOT_FIXED, cpg=cpg))
    return _self(W.concat(pops))


CASES = {
    "quadrupeds+self": lambda: _self(W.quadrupeds(16)),
    "snake3+self": lambda: _self(W.snake(16)),
    "folding chains": _folding_chains,
    "twisted chains": lambda: W.twisted_chains(16),
}


@pytest.mark.parametrize("name, ks", [
    ("quadrupeds+self", [0, 1, 50, 150, 300, 500, 700, 999]),
    ("snake3+self", [0, 1, 100, 300, 600, 900]),
    ("folding chains", [0, 1, 100, 200, 300, 400, 600, 800]),
    ("twisted chains", [0, 1, 100, 250, 400, 550, 700, 850, 999]),
])
def test_self_teacher_forced_one_step(name, ks):
    from paper_2502_11129_amd.sim import Simulator
    pop = CASES[name]()
    _say(f"[self teacher-forced] {name}: {pop.n_variants} variants, steps {ks}")
    sim = Simulator(pop)
    worst, in_band, errs = teacher_forced(pop, sim, ks)
    _say(f"  worst step error {worst:.3e} over {len(errs)} cases; {in_band} in the activation band")
    assert len(errs) > 0
    assert worst <= STEP_TOL


@pytest.mark.parametrize("name, make, T", [
    ("quadrupeds+self x32 T=1000", lambda: _self(W.quadrupeds(32)), 1000),
    ("snake3+self x16 T=1000", lambda: _self(W.snake(16)), 1000),
    ("folding chains x6 T=1000", _folding_chains, 1000),
])
def test_self_fitness_after_T(name, make, T):
    from paper_2502_11129_amd.sim import Simulator
    pop = make()
    _say(f"[self fitness] {name}")
    sim = Simulator(pop)
    sim.rollout(T)
    Fg = sim.fitness().astype(np.float64)
    Fr, F32, Fp, margin = oracle_reference(pop, T)
    _, _, status = sim.counters()
    assert (status == 0).all()
    if pop.root_type == W.ROOT_FIXED:
        # a FIXED root has no displacement: compare the final joint angles instead
        q, _, _ = sim.get_state()
        o = O.Oracle(pop)
        o.step(T, THREADS)
        qr = o.get_state()[0]
        assert np.abs(q - qr).max() < 0.05
    else:
        assert_gate(Fg, Fr, F32, Fp, say=_say, margin=margin)


def test_edge_contacts_teacher_forced():
    """Steps at which the oracle has edge-edge contacts (two bricks crossing
    with no corner inside the other), FREE and FIXED twisted chains: one GPU
    step from the oracle's state meets the 1e-4 bar in every compared
    (step, variant) case that carries such a contact.  The other variants of
    those steps (crumpled chains, some of them FP32-sensitive: the float
    oracle itself misses 1e-4 there) are counted, not held to the bar; the
    other self-collision tests cover them."""
    from paper_2502_11129_amd.sim import Simulator
    total, worst_edge = 0, 0.0
    for root in (W.ROOT_FREE, W.ROOT_FIXED):
        pop = W.twisted_chains(16, root_type=root)
        o = O.Oracle(pop)
        edge = {}
        for k in range(0, 1000, 5):
            q, _, _, _ = o.get_state()
            for i in range(pop.n_variants):
                n = int((o.contacts(i, q[o.q_off[i]:o.q_off[i + 1]])["corner"] == -3).sum())
                if n:
                    edge[(k, i)] = n
            o.step(5, THREADS)
        steps = sorted({k for k, _ in edge})
        ks = steps[:: max(1, len(steps) // 24)][:24]
        _say(f"[edge contacts] twisted chains (root {'FREE' if root == W.ROOT_FREE else 'FIXED'}): "
             f"{len(edge)} (step, variant) states with edge-edge contacts over {len(steps)} steps; steps {ks}")
        worst, in_band, errs, where = teacher_forced(pop, Simulator(pop), ks, keys=True)
        e_edge = np.array([e for e, w in zip(errs, where) if w in edge])
        _say(f"  {len(e_edge)} compared cases with edge-edge contacts, worst step error "
             f"{(e_edge.max() if len(e_edge) else 0.0):.3e}; all {len(errs)} compared cases: worst {worst:.3e}; "
             f"{in_band} in the activation band")
        total += len(e_edge)
        worst_edge = max(worst_edge, float(e_edge.max()) if len(e_edge) else 0.0)
    assert total >= 8
    assert worst_edge <= STEP_TOL


def test_face_contacts_teacher_forced():
    """Steps at which the oracle has face contacts (an edge or face of one
    brick pushed through another's face with no corner inside: the clipped
    incident face), twisted chains whose bricks' rest orientations are tilted
    by up to 0.12 rad so that faces are not exactly coplanar: one GPU step
    from the oracle's state meets the 1e-4 bar in every compared (step,
    variant) case that carries such contacts, the cases near a switch of the
    clip (a candidate at the edge of its validity, the reference or incident
    face choice, the edge-or-face decision) excluded by the activation band.
    Where the float32 instance of the oracle itself misses the bar at the
    same state (stiff, many-row states), the kernel is held to 3x the float
    oracle's error (the FP32-sensitive rule of the fitness gate)."""
    from paper_2502_11129_amd.sim import Simulator
    total, worst_face, by_rule = 0, 0.0, 0
    for root in (W.ROOT_FREE, W.ROOT_FIXED):
        pop = W.tilted(W.twisted_chains(16, root_type=root), 5)
        o = O.Oracle(pop)
        face = {}
        for k in range(0, 1000, 5):
            q, _, _, _ = o.get_state()
            for i in range(pop.n_variants):
                n = int((o.contacts(i, q[o.q_off[i]:o.q_off[i + 1]])["corner"] == -4).sum())
                if n:
                    face[(k, i)] = n
            o.step(5, THREADS)
        steps = sorted({k for k, _ in face})
        ks = steps[:: max(1, len(steps) // 24)][:24]
        _say(f"[face contacts] tilted twisted chains (root {'FREE' if root == W.ROOT_FREE else 'FIXED'}): "
             f"{len(face)} (step, variant) states with face contacts over {len(steps)} steps; steps {ks}")
        worst, in_band, errs, where = teacher_forced(pop, Simulator(pop), ks, keys=True)
        _, _, errs32, where32 = teacher_forced(pop, FloatOracleSim(pop), ks, keys=True)
        e32 = dict(zip(where32, errs32))
        cases = [(e, w) for e, w in zip(errs, where) if w in face]
        bars = np.array([max(STEP_TOL, 3.0 * e32.get(w, 0.0)) for _, w in cases])
        e_face = np.array([e for e, _ in cases])
        over = e_face > STEP_TOL
        _say(f"  {len(e_face)} compared cases with face contacts, worst step error "
             f"{(e_face.max() if len(e_face) else 0.0):.3e}, {int(over.sum())} above 1e-4 where the float oracle's own "
             f"errors are {[f'{e32.get(w, 0.0):.1e}' for (e, w), o in zip(cases, over) if o]}; all {len(errs)} "
             f"compared cases: worst {worst:.3e}; {in_band} in the activation band")
        assert (e_face <= bars).all()
        total += len(e_face)
        by_rule += int(over.sum())
        worst_face = max(worst_face, float(e_face[~over].max()) if (~over).any() else 0.0)
    assert total >= 16
    assert by_rule <= 0.25 * total
    assert worst_face <= STEP_TOL


def test_self_overflow_contacts_bitwise_equal_register_path():
    from paper_2502_11129_amd.sim import Simulator
    pop = _self(W.snake(9))
    _say("[self overflow] snake3+self x9, 2 contacts in registers vs 8, T=1000")
    a = Simulator(pop)
    b = Simulator(pop, contacts_in_registers=2)
    assert [x[2] for x in a.bins()] == [8] and [x[2] for x in b.bins()] == [2]
    a.rollout(1000)
    b.rollout(1000)
    qa, va, _ = a.get_state()
    qb, vb, _ = b.get_state()
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(va, vb)
