"""Closed forms rerun through the GPU kernels (not only through the oracle):
soft-contact rest penetration of a non-cubic box, the contact's damping
rate, Coulomb sliding at mu g, sticking and slipping on an incline, the
implicit PD law settling on its target, and the torque clamp applying
exactly tau_max.  Bars are the oracle pins' bars, widened only where
float32 rounding of the state limits them."""
import sys

import numpy as np
import pytest

from paper_2502_11129_amd import workloads as W

pytestmark = pytest.mark.gpu

G = 9.81
DT = 0.002


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _params(**kw):
    p = dict(W.DEFAULT_PARAMS)
    p.update(kw)
    return p


def _qrot(q):
    w, x, y, z = (float(c) for c in q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _settled_box(half, mu=1.0, t=0.6, g=(0, 0, -G), K=8):
    from paper_2502_11129_amd.sim import Simulator
    pop = W.single_box(half=half, pos=(0, 0, half[2]), mu=mu, params=_params(pgs_iters=K, gravity=g))
    sim = Simulator(pop)
    sim.step(int(round(t / DT)))
    return pop, sim


def test_rest_penetration_of_a_non_cubic_box():
    """Four corners on the plane: the box sinks by g (1 + 3 hy^2 / (hy^2 +
    hz^2) + 3 hx^2 / (hx^2 + hz^2)) / (4 k); with the fixed 8 sweeps within
    5 % (the oracle's bar at K = 8)."""
    hx, hy, hz = 0.1, 0.04, 0.07
    k = W.DEFAULT_PARAMS["k_contact"]
    d_exact = G * (1 + 3 * hy * hy / (hy * hy + hz * hz) + 3 * hx * hx / (hx * hx + hz * hz)) / (4 * k)
    _, sim = _settled_box((hx, hy, hz))
    q, v, _ = sim.get_state()
    R = _qrot(q[3:7])
    d = hz * abs(R[2, 2]) + hx * abs(R[2, 0]) + hy * abs(R[2, 1]) - q[2]   # deepest support below z = 0
    _say(f"[rest] depth {d:.4e} against {d_exact:.4e}")
    assert abs(d - d_exact) / d_exact < 0.05
    assert np.abs(v).max() < 1e-3


def test_contact_damping_rate():
    """After a small vertical kick the resting cube's height decays at
    zeta w0 = 50 /s with half-period pi / (w0 sqrt(1 - zeta^2)) = 36.3 ms."""
    _, sim = _settled_box((0.05, 0.05, 0.05), K=200)
    q, v, k = sim.get_state()
    z_eq = float(q[2])
    v = v.copy()
    v[5] = -0.02                        # body-frame z of an upright cube
    sim.set_state(q, v, k)
    z = []
    for _ in range(100):
        sim.step(1)
        z.append(float(sim.get_state()[0][2]) - z_eq)
    z = np.abs(np.array(z))
    peaks = [i for i in range(1, 99) if z[i] > z[i - 1] and z[i] >= z[i + 1] and z[i] > 1e-7]
    assert len(peaks) >= 2
    rate = np.log(z[peaks[0]] / z[peaks[1]]) / ((peaks[1] - peaks[0]) * DT)
    _say(f"[damping] rate {rate:.1f} /s, half-period {(peaks[1] - peaks[0]) * DT * 1e3:.1f} ms")
    assert 45.0 < rate < 60.0
    assert abs((peaks[1] - peaks[0]) * DT - np.pi / (100 * np.sqrt(0.75))) < 0.006


def test_sliding_box_decelerates_at_mu_g():
    """1 m/s along x on the plane: deceleration mu g and the stopping distance
    v0^2 / (2 mu g) - v0 dt / 2 of semi-implicit Euler, within 1 %."""
    mu, v0 = 0.5, 1.0
    _, sim = _settled_box((0.05, 0.05, 0.05), mu=mu)
    q, v, k = sim.get_state()
    x0 = float(q[0])
    R = _qrot(q[3:7])
    v = v.copy()
    v[3:6] = R.T @ np.array([v0, 0.0, 0.0])
    v[0:3] = 0.0
    sim.set_state(q, v, k)
    xs, vs = [], []
    for _ in range(200):
        sim.step(1)
        qq, vv, _ = sim.get_state()
        xs.append(float(qq[0]) - x0)
        vs.append((_qrot(qq[3:7]) @ vv[3:6].astype(np.float64))[0])
    xs, vs = np.array(xs), np.array(vs)
    d_exact = v0 * v0 / (2 * mu * G) - v0 * DT / 2
    slope = np.polyfit(np.arange(20, 60) * DT, vs[20:60], 1)[0]
    _say(f"[sliding] distance {xs[-1]:.5f} m against {d_exact:.5f}; deceleration {-slope:.4f} against {mu * G:.4f}")
    assert abs(xs[-1] - d_exact) / d_exact < 0.01
    assert abs(vs[-1]) < 1e-3
    assert abs(-slope - mu * G) / (mu * G) < 0.01


def test_incline_stick_and_slip():
    """Gravity tilted by 30 degrees: mu = 1 sticks (creep below 1e-4 m in
    1 s), mu = 0.3 slides at g (sin a - mu cos a) within 1 %."""
    from paper_2502_11129_amd.sim import Simulator
    a = np.radians(30.0)
    g = (G * np.sin(a), 0.0, -G * np.cos(a))
    _, sim = _settled_box((0.05, 0.05, 0.05), mu=1.0, t=0.3, g=g)
    x0 = float(sim.get_state()[0][0])
    sim.step(500)
    creep = abs(float(sim.get_state()[0][0]) - x0)
    acc_exact = G * (np.sin(a) - 0.3 * np.cos(a))
    sim = Simulator(W.single_box(pos=(0, 0, 0.05), mu=0.3, params=_params(gravity=g)))
    sim.step(100)
    x1 = float(sim.get_state()[0][0])
    sim.step(250)
    x2 = float(sim.get_state()[0][0])
    sim.step(250)
    x3 = float(sim.get_state()[0][0])
    acc = ((x3 - x2) - (x2 - x1)) / (0.5 ** 2)
    _say(f"[incline] creep {creep:.2e} m at mu = 1; acceleration {acc:.4f} against {acc_exact:.4f} at mu = 0.3")
    assert creep < 1e-4
    assert abs(acc - acc_exact) / acc_exact < 0.01


def _horizontal_hinge(A, phi):
    """Fixed core, one brick on +x with a vertical hinge axis: gravity exerts no
    torque about it, so the hinge sees only the actuator (target A sin(phi))."""
    return W.chain(1, ["+x"], [W.AXIS_Z], root_type=W.ROOT_FIXED, root_pose=(0, 0, 1.0, 1, 0, 0, 0),
                   theta0=[0.0], cpg=[(A, 0.0, phi)], params=_params())


def test_pd_reaches_target_unclamped():
    from paper_2502_11129_amd.sim import Simulator
    sim = Simulator(_horizontal_hinge(0.1, np.pi / 2))
    sim.step(500)
    q, v, _ = sim.get_state()
    _, clamp, _ = sim.counters()
    _say(f"[pd] theta {q[0]:.8f} against 0.1, thetadot {v[0]:.2e}")
    assert abs(float(q[0]) - 0.1) < 2e-7 and abs(float(v[0])) < 1e-5
    assert clamp[0] == 0


def test_pd_clamp_applies_exactly_tau_max():
    """Large error: the clamp row makes the applied torque tau_max, so the
    hinge spins up at tau_max / I_p, I_p = 5 m h^2 / 3 about the hinge (two
    steps, before kp err - b_a thetadot falls below tau_max)."""
    from paper_2502_11129_amd.sim import Simulator
    sim = Simulator(_horizontal_hinge(1.0, np.pi / 2))
    m, h = np.float32(W.BRICK_MASS), np.float32(W.BRICK_HALF)
    Ip = 5.0 / 3.0 * float(m) * float(h) ** 2
    tmax = W.DEFAULT_PARAMS["tau_max"]
    for n in range(1, 3):
        sim.step(1)
        _, v, _ = sim.get_state()
        want = n * DT * tmax / Ip
        _say(f"[clamp] step {n}: thetadot {v[0]:.7f} against {want:.7f}")
        assert abs(float(v[0]) - want) < 1e-5 * want
    _, clamp, _ = sim.counters()
    assert clamp[0] == 2
