"""Closed-form pins of the oracle's time step: discrete free fall, the
compound pendulum, soft-contact rest penetration and its damping, Coulomb
sliding/sticking, the implicit PD law and its torque clamp, and the
convergence of the fixed-iteration solver as the sweep count grows."""
import numpy as np
import pytest

from paper_2502_11129_amd import workloads as W

G = 9.81


def _params(**kw):
    p = dict(W.DEFAULT_PARAMS)
    p.update(kw)
    return p


def _qrot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_discrete_free_fall(oracle_mod):
    """z_n = z0 + n dt vz0 - g dt^2 n(n+1)/2 exactly (velocity first, then position)."""
    dt, vz0, z0 = 0.002, 0.7, 3.0
    pop = W.single_box(pos=(0.0, 0.0, z0), v_b=(0.3, -0.2, vz0), params=_params())
    o = oracle_mod.Oracle(pop, float32_constants=False)
    for n in (1, 10, 300):
        o.reset()
        o.step(n)
        q, v, k, _ = o.get_state()
        zq = np.float32(z0) + n * dt * np.float64(np.float32(vz0)) - G * dt * dt * n * (n + 1) / 2
        assert k[0] == n
        assert abs(q[2] - zq) < 1e-12
        assert abs(q[0] - n * dt * np.float64(np.float32(0.3))) < 1e-13
        np.testing.assert_allclose(q[3:7], [1, 0, 0, 0], atol=1e-15)


def test_compound_pendulum_period(oracle_mod):
    """Brick on a fixed core, hinge axis y so it hangs at theta = pi/2; small
    swing about the bottom: T = 2 pi sqrt(I_p / (m g l)) with I_p = 5 m h^2 / 3."""
    th_eq = np.pi / 2
    pop = W.chain(1, ["+x"], [W.AXIS_Y], root_type=W.ROOT_FIXED, root_pose=(0, 0, 1.0, 1, 0, 0, 0),
                  theta0=[th_eq + 0.01], params=_params(kp=0.0, kd=0.0))
    o = oracle_mod.Oracle(pop, float32_constants=False)
    m, h = W.BRICK_MASS, W.BRICK_HALF
    T_exact = 2 * np.pi * np.sqrt((5.0 / 3.0 * m * h * h) / (m * G * h))
    assert abs(T_exact - 0.44857) < 1e-5
    n = int(20.5 * T_exact / 0.002)
    th = np.zeros(n)
    for i in range(n):
        o.step(1)
        th[i] = o.get_state()[0][0]
    x = th - th_eq
    up = np.where((x[:-1] < 0) & (x[1:] >= 0))[0]
    t_cross = (up + 1 - x[up + 1] / (x[up + 1] - x[up])) * 0.002   # linear interpolation of crossings
    period = np.diff(t_cross).mean()
    assert len(up) >= 19
    assert abs(period - T_exact) / T_exact < 1e-3


def _settle_box(oracle_mod, half, K=8, mu=1.0, t=0.6, g=(0, 0, -G)):
    pop = W.single_box(half=half, pos=(0, 0, half[2]), mu=mu, params=_params(pgs_iters=K, gravity=g))
    o = oracle_mod.Oracle(pop, float32_constants=False)
    o.step(int(round(t / 0.002)))
    return pop, o


def _mean_depth(o, pop):
    q, _, _, _ = o.get_state()
    c = o.contacts(0, q)
    return c["depth"].mean(), len(c["depth"])


@pytest.mark.parametrize("half", [(0.05, 0.05, 0.05), (0.1, 0.04, 0.07)])
def test_rest_penetration_closed_form(oracle_mod, half):
    """Soft rows in acceleration units: a box resting on its four bottom corners
    sinks by d = g (1 + 3hy^2/(hy^2+hz^2) + 3hx^2/(hx^2+hz^2)) / (4k)
    (g/k = 9.81e-4 m for a cube of any size); exact at solver convergence."""
    hx, hy, hz = half
    k = W.DEFAULT_PARAMS["k_contact"]
    d_exact = G * (1 + 3 * hy * hy / (hy * hy + hz * hz) + 3 * hx * hx / (hx * hx + hz * hz)) / (4 * k)
    pop, o = _settle_box(oracle_mod, half, K=1000)
    d, nc = _mean_depth(o, pop)
    assert nc == 4
    assert abs(d - d_exact) / d_exact < 1e-6
    pop, o = _settle_box(oracle_mod, half, K=8)
    d8, nc = _mean_depth(o, pop)
    assert nc == 4 and abs(d8 - d_exact) / d_exact < 0.05


def test_contact_damping_rate(oracle_mod):
    """The vertical mode of a cube on its four corners is the per-row oscillator
    z'' = -k z - b z' (w0 = 100 rad/s, zeta = 0.5): after a small kick its
    envelope decays at zeta*w0 = 50 /s (loose bound: the implicit step damps a
    little more at w0*dt = 0.2)."""
    pop, o = _settle_box(oracle_mod, (0.05, 0.05, 0.05), K=200)
    q, v, k, _ = o.get_state()
    z_eq = q[2]
    v = v.copy()
    v[5] = -0.02
    o.set_state(q, v, k)
    z = []
    for _ in range(100):
        o.step(1)
        z.append(o.get_state()[0][2] - z_eq)
    z = np.abs(np.array(z))
    peaks = [i for i in range(1, 99) if z[i] > z[i - 1] and z[i] >= z[i + 1] and z[i] > 1e-9]
    assert len(peaks) >= 2
    rate = np.log(z[peaks[0]] / z[peaks[1]]) / ((peaks[1] - peaks[0]) * 0.002)
    assert 45.0 < rate < 60.0, rate
    # half-period between successive |z| peaks: pi / (w0 sqrt(1 - zeta^2)) = 36.3 ms
    half_period = (peaks[1] - peaks[0]) * 0.002
    assert abs(half_period - np.pi / (100 * np.sqrt(0.75))) < 0.006


def test_sliding_box_decelerates_at_mu_g(oracle_mod):
    """From rest on the plane, give a cube 1 m/s along x: it decelerates at mu g
    and stops after v0^2 / (2 mu g) - v0 dt / 2 (the continuous distance less the
    first-order term of semi-implicit Euler), within 1 %."""
    mu, v0 = 0.5, 1.0
    pop, o = _settle_box(oracle_mod, (0.05, 0.05, 0.05), mu=mu)
    q, v, k, _ = o.get_state()
    x0 = q[0]
    R = _qrot(q[3:7])
    v = v.copy()
    v[3:6] = R.T @ np.array([v0, 0.0, 0.0])
    v[0:3] = 0.0
    o.set_state(q, v, k)
    xs, vs = [], []
    for _ in range(200):
        o.step(1)
        qq, vv, _, _ = o.get_state()
        xs.append(qq[0] - x0)
        vs.append((_qrot(qq[3:7]) @ vv[3:6])[0])
    xs, vs = np.array(xs), np.array(vs)
    d_exact = v0 * v0 / (2 * mu * G) - v0 * 0.002 / 2
    assert abs(xs[-1] - d_exact) / d_exact < 0.01
    assert abs(vs[-1]) < 1e-3
    slope = np.polyfit(np.arange(20, 60) * 0.002, vs[20:60], 1)[0]
    assert abs(-slope - mu * G) / (mu * G) < 0.01


def test_incline_stick_and_slip(oracle_mod):
    """Gravity tilted by 30 deg: mu = 1 sticks (tan 30 < 1, creep < 1e-4 m in 1 s),
    mu = 0.3 slides at g (sin a - mu cos a) = 2.356 m/s^2."""
    a = np.radians(30.0)
    g = (G * np.sin(a), 0.0, -G * np.cos(a))
    pop, o = _settle_box(oracle_mod, (0.05, 0.05, 0.05), mu=1.0, t=0.3, g=g)
    x0 = o.get_state()[0][0]
    o.step(500)
    assert abs(o.get_state()[0][0] - x0) < 1e-4
    acc_exact = G * (np.sin(a) - 0.3 * np.cos(a))
    assert abs(acc_exact - 2.356) < 1e-3
    pop = W.single_box(pos=(0, 0, 0.05), mu=0.3, params=_params(gravity=g))
    o = oracle_mod.Oracle(pop, float32_constants=False)
    o.step(100)
    x1 = o.get_state()[0][0]
    o.step(250)
    x2 = o.get_state()[0][0]
    o.step(250)
    x3 = o.get_state()[0][0]
    acc = ((x3 - x2) - (x2 - x1)) / (0.5 ** 2)
    assert abs(acc - acc_exact) / acc_exact < 0.01


def _horizontal_hinge(A, phi, theta0=0.0, **prm):
    """Fixed core, one brick on +x with a vertical hinge axis: gravity exerts no
    torque about it, so the hinge sees only the actuator (target A sin(phi))."""
    return W.chain(1, ["+x"], [W.AXIS_Z], root_type=W.ROOT_FIXED, root_pose=(0, 0, 1.0, 1, 0, 0, 0),
                   theta0=[theta0], cpg=[(A, 0.0, phi)], params=_params(**prm))


def test_pd_reaches_target_unclamped(oracle_mod):
    """Small error (kp*err < tau_max): the implicit PD settles exactly on the target."""
    pop = _horizontal_hinge(0.1, np.pi / 2)
    o = oracle_mod.Oracle(pop, float32_constants=False)
    o.step(500)
    q, v, _, _ = o.get_state()
    assert abs(q[0] - np.float32(0.1)) < 1e-9 and abs(v[0]) < 1e-9
    _, b = o.counters()
    assert b[0] == 0                                   # the clamp never engaged


def test_pd_clamp_applies_exactly_tau_max(oracle_mod):
    """Large error: the clamp row makes the applied torque exactly tau_max, so the
    hinge spins up at tau_max / I_p with I_p = 5 m h^2 / 3 about the hinge
    (for two steps: by then kp * err - b_a * thetadot is back below tau_max)."""
    pop = _horizontal_hinge(1.0, np.pi / 2)
    o = oracle_mod.Oracle(pop, float32_constants=False)
    m, h = W.BRICK_MASS, W.BRICK_HALF
    Ip = 5.0 / 3.0 * np.float64(np.float32(m)) * np.float64(np.float32(h)) ** 2
    tmax, dt = 0.9, 0.002
    for n in range(1, 3):
        o.step(1)
        q, v, _, _ = o.get_state()
        assert abs(v[0] - n * dt * tmax / Ip) < 1e-9 * n * dt * tmax / Ip
    _, b = o.counters()
    assert b[0] == 2


def test_solver_converges_with_sweeps(oracle_mod):
    """One step from a many-contact state: the result converges as the sweep
    count grows (cauchy sequence in K), and K=8 is within a few percent."""
    pop = W.quadrupeds(4)
    o = oracle_mod.Oracle(pop, float32_constants=False)
    o.step(400)
    q, v, k, _ = o.get_state()
    res = {}
    for K in (8, 64, 512, 2048):
        ok = oracle_mod.Oracle(pop, pgs_iters=K, float32_constants=False)
        ok.set_state(q, v, k)
        ok.step(1)
        res[K] = ok.get_state()[1]
    d1 = np.abs(res[512] - res[2048]).max()
    d0 = np.abs(res[64] - res[2048]).max()
    assert d1 < 1e-3 * d0 or d1 < 1e-10
    assert np.abs(res[8] - res[2048]).max() < 0.05 * max(1.0, np.abs(res[2048]).max())
