"""Host-thread worker of the CPU/GPU split (paper Sec. 6), run here without a
GPU: its single-precision rollouts must match the FP64 oracle to the same
fitness bar as the GPU path."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import sim as S
from paper_2502_11129_amd import workloads as W

from _parity import fitness_gate, perturbed_fitness


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
def test_host_worker_matches_oracle(name, pop, T):
    h = S.Handle(pop)
    Fh, sec = h.rollout_host(T, threads=4)
    Fr = O.Oracle(pop).rollout(T, threads=4)
    F32 = O.Oracle(pop, precision=32).rollout(T, threads=4)
    ok, chaotic, ratio = fitness_gate(Fh.astype(np.float64), Fr, F32, perturbed_fitness(pop, T))
    assert ok.all(), (name, np.where(~ok)[0], Fh[~ok], Fr[~ok], ratio.max())
    assert sec > 0


def test_host_worker_thread_count_does_not_change_results():
    pop = W.random_trees(13)
    h = S.Handle(pop)
    a, _ = h.rollout_host(300, threads=1)
    b, _ = h.rollout_host(300, threads=5)
    np.testing.assert_array_equal(a, b)
