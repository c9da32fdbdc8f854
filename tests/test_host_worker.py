"""Host-thread worker of the CPU/GPU split (paper Sec. 6), run here without a
GPU: its single-precision rollouts must match the FP64 oracle to the same
fitness bar as the GPU path, with either factorisation of the joint-space
system (dense Cholesky, tree-sparse L^T L)."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import sim as S
from paper_2502_11129_amd import workloads as W

from _parity import assert_gate, oracle_reference


@pytest.mark.parametrize("name, pop, T", [
    ("snake3 x16", W.snake(16), 1000),
    ("boxes x64", W.boxes(64), 1000),
    ("trees x24", W.random_trees(24), 600),
    ("quadrupeds x8", W.quadrupeds(8), 400),
    ("fixed chain", W.chain(3, ["+x", "+y", "+x"], [1, 0, 1], theta0=[0.3, -0.2, 0.5],
                            cpg=[(0.8, 3.0, 0.1), (0.5, 2.0, 1.0), (0.9, 4.0, 2.0)]), 500),
    ("box_and_ball x48", W.box_and_ball(48), 1000),
    ("snake3+ball x16", W.attach_ball(W.snake(16)), 800),
    ("quadrupeds+self x16", dataclasses.replace(W.quadrupeds(16), self_collision=True), 800),
])
@pytest.mark.parametrize("factorization", ["dense", "tree"])
def test_host_worker_matches_oracle(name, pop, T, factorization):
    h = S.Handle(pop, host_factorization=factorization)
    Fh, sec = h.rollout_host(T, threads=4)
    Fr, F32, Fp, margin = oracle_reference(pop, T, threads=4)
    assert_gate(Fh.astype(np.float64), Fr, F32, Fp, label=f"{name} {factorization}: ", margin=margin)
    assert sec > 0


def test_host_worker_thread_count_does_not_change_results():
    pop = W.random_trees(13)
    h = S.Handle(pop)
    a, _ = h.rollout_host(300, threads=1)
    b, _ = h.rollout_host(300, threads=5)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("name, pop", [
    ("trees x32", W.random_trees(32)),
    ("box_and_ball x32", W.box_and_ball(32)),
    ("quadrupeds+self x8", dataclasses.replace(W.quadrupeds(8), self_collision=True)),
])
def test_tree_factorization_agrees_with_dense_to_rounding(name, pop):
    """Same system, two factorisations, so the same trajectories up to
    single-precision rounding: over 100 steps the typical fitness difference
    is at rounding level, and the worst (rounding carried through a contact
    or clamp decision) stays below 0.2 mm."""
    F = {}
    for f in ("dense", "tree"):
        F[f], _ = S.Handle(pop, host_factorization=f).rollout_host(100, threads=4)
    assert np.isfinite(F["dense"]).all() and np.isfinite(F["tree"]).all()
    d = np.abs(F["tree"] - F["dense"])
    assert np.median(d) < 1e-6, np.median(d)
    assert d.max() < 2e-4, d.max()


def test_host_factorization_option_is_validated():
    o = S.make_options()
    o.host_factorization = 2
    lib = S.load()
    desc, keep = S.make_desc(W.boxes(2))
    h = S.C.c_void_p()
    assert lib.sim_create(S.C.byref(desc), S.C.byref(o), S.C.byref(h)) == S.SIM_E_INVALID
    assert b"host_factorization" in lib.sim_last_error(None)


def test_autotune_host_returns_a_factorization_and_both_timings():
    from paper_2502_11129_amd.autotune import autotune_host
    best, times = autotune_host(W.random_trees(40), T_pilot=50, threads=2, sample=8)
    assert best in ("dense", "tree") and set(times) == {"dense", "tree"}
    assert times[best] == min(times.values())


def test_tree_factorization_flop_count_closed_forms():
    """The flop count of the tree-sparse factorisation against closed forms:
    a snake is a chain of DoFs (DoF k has k ancestors: 1 + k + k (k + 1)
    flops to factor, 4 k + 2 to solve), a ball's six DoFs are isolated (one
    square root, two divisions each), and a quadruped's DoF tree starts with
    the free root's chain and saves most of the dense work."""
    from paper_2502_11129_amd import flops as FL
    snake = W.snake(1)
    n = int(snake.nv[0])
    fac, sol = FL.factor_solve_flops(snake, "tree")
    assert fac[0] == sum(1 + k + k * (k + 1) for k in range(n))
    assert sol[0] == sum(4 * k + 2 for k in range(n))
    fac_b, sol_b = FL.factor_solve_flops(W.attach_ball(W.snake(1)), "tree")
    assert fac_b[0] == fac[0] + 6 and sol_b[0] == sol[0] + 12
    lam = FL.dof_parents(W.quadrupeds(1), 0)
    assert (lam < np.arange(len(lam))).all()                     # parents come first
    assert list(lam[:6]) == [-1, 0, 1, 2, 3, 4]                  # the free root's chain
    d_fac, _ = FL.factor_solve_flops(W.quadrupeds(1), "dense")
    t_fac, _ = FL.factor_solve_flops(W.quadrupeds(1), "tree")
    assert t_fac[0] < d_fac[0] / 3                               # four limbs: branch-induced sparsity


def test_step_flop_model_switches_to_the_sparse_counts_per_variant():
    """With the tree-sparse factorisation a variant's factorisation and
    solves (free velocity, three per contact, one per clamp) are counted at
    the sparse algorithm's flops; the rest of the step is unchanged."""
    from paper_2502_11129_amd import flops as FL
    pop = W.quadrupeds(4)
    nc, ncl, T = np.array([30, 0, 7, 12]), np.array([5, 0, 2, 9]), 10
    dense = FL.flops_per_variant(pop, T, nc, ncl)
    fac = np.array(["dense", "tree", "tree", "dense"])
    mixed = FL.flops_per_variant(pop, T, nc, ncl, factorization=fac)
    nv = pop.nv.astype(np.float64)
    tf, ts = FL.factor_solve_flops(pop, "tree")
    want = dense - (T * ((2 / 3) * nv ** 3 + 2 * nv ** 2 - tf - ts)
                    + nc * 3 * (2 * nv ** 2 - ts) + ncl * (2 * nv ** 2 - ts))
    np.testing.assert_allclose(mixed[1:3], want[1:3], rtol=1e-12)
    np.testing.assert_array_equal(mixed[[0, 3]], dense[[0, 3]])
