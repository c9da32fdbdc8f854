"""GPU tests of the C ABI's device-side transfers and of re-binding.

sim_get_state / sim_set_state / sim_counters with where = SIM_DEVICE move the
state between the library's packed bins and caller device arrays in the
variant-CSR layout; they must agree with the host path bit for bit.  A second
sim_bind on another workspace must drop a captured rollout graph (which holds
the first workspace's pointers) and run from the new one."""
import sys

import numpy as np
import pytest

from paper_2502_11129_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sim(pop, **kw):
    from paper_2502_11129_amd.sim import Simulator
    return Simulator(pop, **kw)


def test_device_state_transfer_matches_host_path():
    import torch
    pop = W.concat([W.random_trees(37), W.random_trees(5, first=37)])   # several bins, ragged waves
    _say("[boundary] device get/set state and counters, trees x42")
    a = _sim(pop)
    a.step(250)
    q, v, k = a.get_state()
    qd, vd, kd = a.get_state_device()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(qd.cpu().numpy(), q)
    np.testing.assert_array_equal(vd.cpu().numpy(), v)
    np.testing.assert_array_equal(kd.cpu().numpy(), k)
    ca, cb, cs = a.counters()
    da, db, ds = a.counters_device()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(da.cpu().numpy().astype(np.uint64), ca)
    np.testing.assert_array_equal(db.cpu().numpy().astype(np.uint64), cb)
    np.testing.assert_array_equal(ds.cpu().numpy().astype(np.uint32), cs)
    assert ca.max() > 0
    # resume from device arrays in a fresh simulator: same continuation as the original
    b = _sim(pop)
    b.set_state_device(qd, vd, kd)
    a.step(150)
    b.step(150)
    qa, va, ka = a.get_state()
    qb, vb, kb = b.get_state()
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(va, vb)
    np.testing.assert_array_equal(ka, kb)
    # set_state without k keeps the step counters; a frozen variant is cleared
    vbad = vd.clone()
    vbad[int(pop.v_offset[3]) + 6] = float("nan")
    b.set_state_device(qd, vbad)
    assert (b.get_state()[2] == 400).all()
    b.step(1)
    assert b.counters()[2][3] == 1
    b.set_state_device(qd, vd)
    _, _, kk = b.get_state()
    assert kk[3] == 400 and (np.delete(kk, 3) == 401).all()
    assert (b.counters()[2] == 0).all()


def test_rebind_drops_captured_graph():
    import torch
    from paper_2502_11129_amd.sim import SIM_OK
    import ctypes as C
    pop = W.snake(16)
    _say("[boundary] graph rollout, rebind to a new workspace, graph rollout again")
    e = _sim(pop)
    e.rollout(300)
    Fe = e.fitness()
    g = _sim(pop, use_graph=True)
    g.rollout(300)
    np.testing.assert_array_equal(g.fitness(), Fe)
    old = g.ws
    g.ws = torch.empty_like(old)
    assert g.lib.sim_bind(g.h, C.c_void_p(g.ws.data_ptr()), g.ws.numel(), g.stream()) == SIM_OK
    old.fill_(255)               # the first workspace is garbage now; nothing may read it
    torch.cuda.synchronize()
    del old
    for _ in range(2):
        g.rollout(300)
        np.testing.assert_array_equal(g.fitness(), Fe)
