"""Parity at the full benchmark sizes, in the launch configurations bench.py
times: 8192 random trees x 5000 steps (the autotuner's layout: the <= 16-DoF
variants in one two-wave 16-body bin, the 20-DoF ones in the two-wave
16-body kernel with 4 contacts in registers, the larger in 32-body kernels;
and the 32-body layout on four streams),
512 000 box-and-ball variants x 1000 steps, 32 768 quadrupeds x 1000 steps
with and without self-collision, and all 4096 dropped boxes x 2000 steps
against the oracle variant by variant.  The oracle cannot run the larger
populations whole, so their sampled variants are checked two ways: bitwise against the same variants
simulated on their own (a variant's arithmetic does not depend on the other
variants of its wave, bin or launch), and against the FP64 oracle with the
fitness gate of the small-size parity tests."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import workloads as W

from _parity import THREADS, assert_gate, oracle_reference

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(pop, T, **opts):
    from paper_2502_11129_amd.sim import Simulator
    sim = Simulator(pop, **opts)
    sim.rollout(T)
    F = sim.fitness()
    q, v, k = sim.get_state()[:3]
    status = sim.counters()[2]
    sim.close()
    return F, np.asarray(q), np.asarray(v), np.asarray(k), status


def _rows(pop, idx, q, v):
    """The listed variants' state entries out of whole-population arrays."""
    qo, vo = pop.q_offset, pop.v_offset
    qs = np.concatenate([q[qo[i]:qo[i + 1]] for i in idx])
    vs = np.concatenate([v[vo[i]:vo[i + 1]] for i in idx])
    return qs, vs


@pytest.mark.parametrize("name, make, T, opts, sample", [
    ("trees 8192 x 5000", lambda: W.random_trees(8192), 5000,
     dict(min_body_slots=32, slots32_min_nvc=24, min_nv_capacity=16, ncr_by_nvc={16: 8, 20: 4}),
     np.array(W.TREE_SPOTCHECK)),
    ("trees 8192 x 5000, 32-body kernels on four streams", lambda: W.random_trees(8192), 5000,
     dict(min_body_slots=32, streams=4), np.array(W.TREE_SPOTCHECK)),
    ("box_and_ball 512000 x 1000", lambda: W.box_and_ball(512000), 1000, dict(),
     np.arange(0, 512000, 8000)),
    ("quadrupeds+self 32768 x 1000", lambda: dataclasses.replace(W.quadrupeds(32768), self_collision=True), 1000,
     dict(min_body_slots=32), np.arange(0, 32768, 2048)),
    ("quadrupeds 32768 x 1000", lambda: W.quadrupeds(32768), 1000, dict(), np.arange(0, 32768, 1024)),
])
def test_full_size_sampled_variants(name, make, T, opts, sample):
    pop = make()
    _say(f"[full size] {name}, options {opts}: {len(sample)} sampled variants")
    F, q, v, k, status = _run(pop, T, **opts)
    assert (status == 0).all()
    sub = pop.subset(sample)
    Fs, qs, vs, ks, _ = _run(sub, T)
    qf, vf = _rows(pop, sample, q, v)
    np.testing.assert_array_equal(F[sample], Fs)
    np.testing.assert_array_equal(qf, qs)
    np.testing.assert_array_equal(vf, vs)
    np.testing.assert_array_equal(k[sample], ks)
    _say("  sampled variants bitwise equal to their own run; oracle ...")
    Fr, F32, Fp, margin = oracle_reference(sub, T)
    assert_gate(Fs.astype(np.float64), Fr, F32, Fp, say=_say, margin=margin)


def test_full_size_boxes_every_variant():
    """The whole box population (4096 free boxes x 2000 steps) against the
    oracle, every variant under the fitness gate."""
    pop = W.boxes(4096)
    T = 2000
    _say(f"[full size] boxes 4096 x {T}: every variant against the oracle")
    F, q, v, k, status = _run(pop, T)
    assert (status == 0).all() and (k == T).all()
    Fr, F32, Fp, margin = oracle_reference(pop, T)
    assert_gate(F.astype(np.float64), Fr, F32, Fp, say=_say, margin=margin)
