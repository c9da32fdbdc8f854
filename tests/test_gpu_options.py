"""Launch and packing options change layout, never results (GPU); the split
pilot leaves the population in its initial state."""
import sys

import numpy as np
import pytest

from paper_2502_11129_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_autotuned_options_run_and_match_the_defaults():
    """The autotuner (coordinate descent from four layouts, then an
    interleaved final round among the near-best) returns options the
    simulator accepts, and they give the default options' results bit for
    bit (with the same factorisation of M~, the one option that changes
    rounding)."""
    from paper_2502_11129_amd.autotune import autotune
    from paper_2502_11129_amd.sim import Simulator
    pop = W.random_trees(512)
    T = 200
    opts, trials = autotune(pop, T_pilot=T, reps=1, log=_say)
    _say(f"[autotune] {len(trials)} trials, chose {opts}")
    assert opts in [t["options"] for t in trials]
    a = Simulator(pop, gpu_factorization=opts.get("gpu_factorization", "dense"))
    b = Simulator(pop, **opts)
    a.rollout(T)
    b.rollout(T)
    np.testing.assert_array_equal(a.fitness(), b.fitness())


def test_options_give_bitwise_identical_results():
    from paper_2502_11129_amd.sim import Simulator
    pop = W.random_trees(indices=W.TREE_SPOTCHECK)
    T = 300
    ref = Simulator(pop)
    ref.rollout(T)
    Fr = ref.fitness()
    qr, vr, kr = ref.get_state()
    for opts in (dict(streams=1), dict(streams=2), dict(steps_per_launch=97), dict(min_body_slots=32),
                 dict(ncr_by_nvc={24: 2, 28: 2, 20: 2}), dict(ncr_by_nvc={28: 12}),
                 dict(min_body_slots=32, single_launch=True),
                 dict(min_body_slots=32, slots32_min_nvc=20, min_nv_capacity=16, ncr_by_nvc={16: 8}),
                 dict(min_body_slots=32, ncr_by_nvc={16: 8}),
                 dict(min_body_slots=32, slots32_min_nvc=24, min_nv_capacity=16, ncr_by_nvc={16: 8, 20: 2}),
                 dict(min_body_slots=32, slots32_min_nvc=24, min_nv_capacity=16, ncr_by_nvc={16: 8, 20: 4}),
                 dict(min_body_slots=32, single_launch=True, steps_per_launch=70)):
        _say(f"[options] {opts}")
        s = Simulator(pop, **opts)
        s.rollout(T)
        q, v, k = s.get_state()
        np.testing.assert_array_equal(s.fitness(), Fr)
        np.testing.assert_array_equal(q, qr)
        np.testing.assert_array_equal(v, vr)
        np.testing.assert_array_equal(k, kr)


def test_plan_split_measures_and_resets():
    from paper_2502_11129_amd.sim import Simulator
    pop = W.quadrupeds(512)
    s = Simulator(pop)
    s.step(50)
    plan = s.plan_split(T_pilot=50, threads=4, host_sample=16)
    _say(f"[plan] {plan}")
    assert len(plan["gpu_n"]) >= 3 and plan["gpu_n"][-1] == 512
    assert all(b > a for a, b in zip(plan["gpu_n"], plan["gpu_n"][1:]))
    assert all(t > 0 for t in plan["gpu_s"]) and plan["host_s_per_variant"] > 0
    assert 0 <= plan["n_host_makespan"] <= 512 and 0 <= plan["n_host_paper"] <= 512
    assert plan["makespan_opt_s"] <= plan["makespan_paper_s"] + 1e-12
    q, v, k = s.get_state()
    assert (k == 0).all()
    np.testing.assert_array_equal(q, pop.q0.astype(np.float32))
    np.testing.assert_array_equal(v, pop.v0.astype(np.float32))


def test_rollout_in_chunks_matches_one_handle():
    """A population run as consecutive chunks that each fit a workspace cap
    (a fifth of the whole) gives every variant the fitness, counters and
    status of one handle over the whole population, bit for bit."""
    from paper_2502_11129_amd.sim import Handle, Simulator, rollout_in_chunks
    pop = W.random_trees(300)
    T = 300
    whole = Simulator(pop)
    whole.rollout(T)
    a, b, s = whole.counters()
    cap = Handle(pop).workspace_bytes() // 5
    r = rollout_in_chunks(pop, T, max_workspace_bytes=cap)
    _say(f"[chunks] cap {cap} bytes: chunk ends {r['chunks']}")
    assert len(r["chunks"]) >= 5
    np.testing.assert_array_equal(r["fitness"], whole.fitness())
    np.testing.assert_array_equal(r["rows_contact"], a)
    np.testing.assert_array_equal(r["rows_clamp"], b)
    np.testing.assert_array_equal(r["status"], s)
