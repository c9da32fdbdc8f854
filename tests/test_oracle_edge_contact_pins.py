"""Pins of the oracle's edge-edge box contact (two edges crossing with no
corner of either box inside the other), against closed forms and brute force.

* Closed form: box P turned 45 deg about x (its lowest edge runs along x),
  box Q turned 45 deg about y (its highest edge runs along y) below it, the
  two edges pushed delta into each other: one contact at the crossing,
  normal +z, depth delta, for cubes and for general half extents; the same
  after any rigid motion of the pair; swapping the boxes flips the normal.
* Brute force on perturbed crossings: the depth is the least overlap of the
  two boxes over a dense sampling of all directions (the boxes' corner
  support functions), the normal is that direction, and the point is the
  midpoint of the closest points of the two edges found by a grid search.
* No contact when the boxes are apart or when the least overlap is along a
  face normal."""
import numpy as np
import pytest

from oracle import oracle as O


def _rx(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def _ry(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _rz(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _random_rotation(rng):
    q = rng.normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _crossing(hP, hQ, delta):
    """P turned 45 deg about x at the origin, Q turned 45 deg about y below
    it with the two edges overlapping by delta; the expected contact."""
    s2 = np.sqrt(2.0)
    lowP = (hP[1] + hP[2]) / s2      # depth of P's lowest edge below its centre
    highQ = (hQ[0] + hQ[2]) / s2     # height of Q's highest edge above its centre
    pQ = np.array([0.0, 0.0, -lowP - highQ + delta])
    # P's lowest edge is its local edge (y, z) = (-hy, -hz), at world y = (hz - hy) / sqrt 2;
    # Q's highest edge is its local edge (x, z) = (-hx, +hz), at world x = (hz - hx) / sqrt 2
    x = np.array([(hQ[2] - hQ[0]) / s2, (hP[2] - hP[1]) / s2, -lowP + delta / 2])
    return (np.zeros(3), _rx(np.pi / 4), np.asarray(hP, float), pQ, _ry(np.pi / 4), np.asarray(hQ, float),
            x, np.array([0.0, 0.0, 1.0]), delta)


def _corners(p, R, h):
    s = np.array([[(c & 1) * 2 - 1, ((c >> 1) & 1) * 2 - 1, ((c >> 2) & 1) * 2 - 1] for c in range(8)], float)
    return p + (s * h) @ R.T


def _inside(x, p, R, h):
    return bool(np.all(np.abs(R.T @ (x - p)) < h))


@pytest.mark.parametrize("hP, hQ", [((0.05, 0.05, 0.05), (0.05, 0.05, 0.05)),
                                    ((0.08, 0.03, 0.05), (0.02, 0.07, 0.04)),
                                    ((0.06, 0.03, 0.03), (0.05, 0.1, 0.06))])
@pytest.mark.parametrize("delta", [1e-4, 2e-3, 8e-3])
def test_crossing_edges_closed_form(hP, hQ, delta):
    pP, RP, hp, pQ, RQ, hq, x, n, d = _crossing(hP, hQ, delta)
    for c in _corners(pP, RP, hp):
        assert not _inside(c, pQ, RQ, hq)
    for c in _corners(pQ, RQ, hq):
        assert not _inside(c, pP, RP, hp)
    r = O.edge_contact(pP, RP, hp, pQ, RQ, hq)
    assert r is not None
    np.testing.assert_allclose(r[0], x, atol=1e-12)
    np.testing.assert_allclose(r[1], n, atol=1e-12)
    assert abs(r[2] - d) <= 1e-12
    # a rigid motion of the pair moves the contact with it; swapping flips the normal
    rng = np.random.default_rng(int(delta * 1e6) + len(hP))
    G, t = _random_rotation(rng), rng.normal(size=3)
    r2 = O.edge_contact(G @ pP + t, G @ RP, hp, G @ pQ + t, G @ RQ, hq)
    np.testing.assert_allclose(r2[0], G @ x + t, atol=1e-12)
    np.testing.assert_allclose(r2[1], G @ n, atol=1e-12)
    assert abs(r2[2] - d) <= 1e-12
    r3 = O.edge_contact(pQ, RQ, hq, pP, RP, hp)
    np.testing.assert_allclose(r3[0], x, atol=1e-12)
    np.testing.assert_allclose(r3[1], -n, atol=1e-12)
    assert abs(r3[2] - d) <= 1e-12


def _fibonacci_sphere(m):
    i = np.arange(m) + 0.5
    phi = np.arccos(1 - 2 * i / m)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def _closest_on_edges(a0, a1, b0, b1):
    """Closest points of segments a0-a1 and b0-b1 by nested grid search."""
    lo = np.array([0.0, 0.0])
    hi = np.array([1.0, 1.0])
    for _ in range(6):
        ts = np.linspace(lo[0], hi[0], 201)
        ss = np.linspace(lo[1], hi[1], 201)
        A = a0 + ts[:, None] * (a1 - a0)
        B = b0 + ss[:, None] * (b1 - b0)
        D = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
        i, j = np.unravel_index(np.argmin(D), D.shape)
        wt, ws = (hi[0] - lo[0]) / 20, (hi[1] - lo[1]) / 20
        lo = np.array([max(0.0, ts[i] - wt), max(0.0, ss[j] - ws)])
        hi = np.array([min(1.0, ts[i] + wt), min(1.0, ss[j] + ws)])
    return A[i], B[j]


def test_perturbed_crossings_against_brute_force():
    rng = np.random.default_rng(7)
    dirs = _fibonacci_sphere(200000)
    checked = 0
    for trial in range(60):
        hP = rng.uniform(0.02, 0.08, 3)
        hQ = rng.uniform(0.02, 0.08, 3)
        pP, RP, hp, pQ, RQ, hq, _, _, _ = _crossing(hP, hQ, rng.uniform(5e-4, 4e-3))
        Gp, Gq = _rx(rng.uniform(-0.15, 0.15)) @ _rz(rng.uniform(-0.15, 0.15)), _ry(rng.uniform(-0.15, 0.15))
        RP, RQ = Gp @ RP, Gq @ RQ
        pQ = pQ + rng.normal(0, 0.002, 3)
        cP, cQ = _corners(pP, RP, hp), _corners(pQ, RQ, hq)
        if any(_inside(c, pQ, RQ, hq) for c in cP) or any(_inside(c, pP, RP, hp) for c in cQ):
            continue
        r = O.edge_contact(pP, RP, hp, pQ, RQ, hq)
        if r is None:
            continue
        x, n, depth = r
        # least overlap over all directions: support of Q along u minus the lowest of P along u
        ov = (cQ @ dirs.T).max(0) - (cP @ dirs.T).min(0)
        u0 = dirs[np.argmin(ov)]
        # refine in a cap of 0.03 rad around the best sample
        t1 = np.cross(u0, [1.0, 0.0, 0.0] if abs(u0[0]) < 0.9 else [0.0, 1.0, 0.0])
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(u0, t1)
        a, b = np.meshgrid(np.linspace(-0.03, 0.03, 601), np.linspace(-0.03, 0.03, 601))
        loc = u0 + a.reshape(-1, 1) * t1 + b.reshape(-1, 1) * t2
        loc /= np.linalg.norm(loc, axis=1, keepdims=True)
        ovl = (cQ @ loc.T).max(0) - (cP @ loc.T).min(0)
        assert min(ov.min(), ovl.min()) >= depth - 1e-12   # no direction overlaps less
        assert ovl.min() <= depth + 1e-5                    # sampling resolution
        assert np.dot(loc[np.argmin(ovl)], n) > 0.9999
        ovn = (cQ @ n).max() - (cP @ n).min()
        assert abs(ovn - depth) <= 1e-12
        # the edges: P's corners lowest along n, Q's highest along n (two of each)
        eP = cP[np.argsort(cP @ n)[:2]]
        eQ = cQ[np.argsort(-(cQ @ n))[:2]]
        a, b = _closest_on_edges(eP[0], eP[1], eQ[0], eQ[1])
        np.testing.assert_allclose(x, 0.5 * (a + b), atol=2e-6)
        checked += 1
    assert checked >= 30


def test_no_contact_when_apart_or_face_axis_least():
    pP, RP, hp, pQ, RQ, hq, _, _, _ = _crossing((0.05,) * 3, (0.05,) * 3, -1e-3)   # edges 1 mm apart
    assert O.edge_contact(pP, RP, hp, pQ, RQ, hq) is None
    # two axis-aligned boxes overlapping face to face: least overlap along a face normal
    I = np.eye(3)
    assert O.edge_contact([0, 0, 0], I, [0.05] * 3, [0, 0, -0.099], I, [0.05] * 3) is None
