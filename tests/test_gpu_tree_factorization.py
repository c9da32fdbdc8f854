"""The rollout kernel with the tree-sparse factorisation of M~ (GPU):
M~ = L^T L over the DoF tree, factored in LDS from the last DoF to the first
with no fill-in, and M~^-1 formed by two triangular solves per DoF, in place
of the dense Gauss-Jordan sweep (sim_options.gpu_factorization).  It is held
to the dense kernels' bars against the FP64 oracle: the per-step state error
from the oracle's own states and the fitness gate after T steps."""
import sys

import numpy as np
import pytest

from _parity import STEP_TOL, assert_gate, oracle_reference, teacher_forced
from paper_2502_11129_amd import workloads as W

pytestmark = pytest.mark.gpu

TREE_OPTS = dict(min_body_slots=32, gpu_factorization="tree")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _trees24(n, start=0):
    """Random trees of 15-18 hinges under the free core (21-24 DoFs), the
    shape of the compiled tree-sparse kernel, in index order from `start`."""
    idx, i = [], start
    while len(idx) < n:
        if 15 <= len(W.random_tree(i)[0]) <= 18:
            idx.append(i)
        i += 1
    return W.random_trees(indices=idx)


def test_tree_kernel_is_used_only_where_compiled():
    from paper_2502_11129_amd.sim import Simulator
    pop = W.random_trees(512)
    s = Simulator(pop, **TREE_OPTS)
    fac = s.bin_factorization()
    _say(f"[tree] bins {s.bins()} factorisation {fac}")
    for (nvc, nbc, ncr, _), f in zip(s.bins(), fac):
        assert f == ("tree" if (nvc, nbc, ncr) == (24, 32, 8) else "dense")
    assert "tree" in fac
    assert set(Simulator(pop, min_body_slots=32).bin_factorization()) == {"dense"}
    assert set(Simulator(pop, single_launch=True, **TREE_OPTS).bin_factorization()) == {"dense"}


def test_tree_kernel_teacher_forced_one_step():
    from paper_2502_11129_amd.sim import Simulator
    pop = _trees24(64)
    sim = Simulator(pop, **TREE_OPTS)
    assert sim.bin_factorization() == ["tree"]
    ks = [0, 1, 10, 100, 400, 1000, 2000, 3000, 4999]
    _say(f"[tree teacher-forced] {pop.n_variants} trees of 21-24 DoFs, steps {ks}")
    worst, in_band, errs = teacher_forced(pop, sim, ks)
    _say(f"  worst step error {worst:.3e} over {len(errs)} cases; {in_band} in the activation band")
    assert len(errs) > 400
    assert worst <= STEP_TOL


def test_tree_and_dense_kernels_agree_to_rounding_in_one_step():
    """One step from the same states by both kernels: the factorisations
    differ only in rounding, so the states agree far inside the parity bar."""
    from paper_2502_11129_amd.sim import Simulator
    pop = _trees24(128, start=5000)
    a = Simulator(pop, min_body_slots=32)
    b = Simulator(pop, **TREE_OPTS)
    a.step(700)
    q, v, k = a.get_state()
    b.set_state(q, v, k)
    a.step(1)
    b.step(1)
    qa, va, _ = a.get_state()
    qb, vb, _ = b.get_state()
    dv = np.abs(va.astype(np.float64) - vb) / np.maximum(np.abs(va), 1.0)
    dq = np.abs(qa.astype(np.float64) - qb) / np.maximum(np.abs(qa), 1.0)
    _say(f"[tree vs dense] max relative difference: v {dv.max():.2e}, q {dq.max():.2e}")
    assert dv.max() <= 0.1 * STEP_TOL and dq.max() <= 0.1 * STEP_TOL
    assert dv.max() > 0.0              # a different kernel ran


def test_tree_kernel_fitness_gate():
    from paper_2502_11129_amd.sim import Simulator
    pop = _trees24(256, start=20000)
    T = 2000
    sim = Simulator(pop, **TREE_OPTS)
    assert sim.bin_factorization() == ["tree"]
    sim.rollout(T)
    _, _, st = sim.counters()
    assert (st == 0).all()
    Fg = sim.fitness().astype(np.float64)
    Fr, F32, Fp, margin = oracle_reference(pop, T)
    assert_gate(Fg, Fr, F32, Fp, say=_say, label="tree-sparse kernel", margin=margin)
