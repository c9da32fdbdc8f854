"""Pins of the oracle's face contacts between two boxes (an edge or a face of
one box pushed through a face of the other with no corner of either inside,
the least overlap along a face normal): the incident face clipped to the
reference face.

* Closed form: a long brick lying across a cube's top face, turned by an
  angle about the vertical and sunk delta: four contacts where the brick's
  bottom edges cross the cube's side planes, depth delta, normal +z, on the
  brick; with the boxes swapped, the same four points on the cube's top face,
  normal -z (the brick's face is then the reference, first of equals).
* Rigid motion of the pair moves the contacts with it.
* Brute force: on perturbed crossings the contacts are exactly the vertices
  of the incident face clipped to the reference rectangle by a
  Sutherland-Hodgman pass written here, lifted back onto the incident face,
  that lie below the reference face; the oracle's detect() lists them for a
  robot's boxes.
* No face contact when the boxes are apart or when an edge pair beats every
  face axis by the margin; edges in parallel planes (an edge-pair axis along
  the face normal, the same overlap) stay a face case."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_11129_amd import workloads as W


def _rz(t):
    c, s = np.cos(t), np.sin(t)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _random_rotation(rng):
    q = rng.normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _small_rotation(rng, a):
    w = rng.uniform(-a, a, 3)
    th = np.linalg.norm(w)
    k = w / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def _corners(p, R, h):
    s = np.array([[(c & 1) * 2 - 1, ((c >> 1) & 1) * 2 - 1, ((c >> 2) & 1) * 2 - 1] for c in range(8)], float)
    return p + (s * h) @ R.T


def _inside(x, p, R, h):
    return (np.abs(R.T @ (x - p)) < h).all()


CUBE = 0.05
BRICK = np.array([0.2, 0.02, 0.02])


def _across(theta, delta):
    """Cube at the origin; the brick across its top face, turned theta about z
    and sunk delta."""
    return (np.zeros(3), np.eye(3), np.full(3, CUBE), np.array([0.0, 0.0, CUBE + BRICK[2] - delta]), _rz(theta),
            BRICK.copy())


def _expected_across(theta, delta, z):
    """The crossings of the brick's long bottom edges (offset +-hy across its
    length) with the cube's side planes x = +-h: y = x tan(theta) + o / cos(theta)."""
    pts = []
    for o in (-BRICK[1], BRICK[1]):
        for xs in (-CUBE, CUBE):
            pts.append([xs, xs * np.tan(theta) + o / np.cos(theta), z])
    return np.array(pts)


def _same_set(a, b, tol):
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape:
        return False
    used = set()
    for p in a:
        d = np.linalg.norm(b - p, axis=1)
        j = int(np.argmin(d))
        if d[j] > tol or j in used:
            return False
        used.add(j)
    return True


@pytest.mark.parametrize("theta", [np.radians(10.0), np.radians(-25.0), np.radians(4.0)])
@pytest.mark.parametrize("delta", [1e-3, 4e-3])
def test_brick_across_a_cube_closed_form(theta, delta):
    pP, RP, hP, pQ, RQ, hQ = _across(theta, delta)
    x, d, n, who = O.face_contacts(pP, RP, hP, pQ, RQ, hQ)
    assert who == "Q" and len(x) == 4
    np.testing.assert_allclose(n, [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(d, delta, rtol=0, atol=1e-15)
    assert _same_set(x, _expected_across(theta, delta, CUBE - delta), 1e-14)
    # swapped: the brick's bottom face is the reference (first of equal overlaps)
    x, d, n, who = O.face_contacts(pQ, RQ, hQ, pP, RP, hP)
    assert who == "Q" and len(x) == 4                      # the points now lie on the cube (Q)
    np.testing.assert_allclose(n, [0, 0, -1], atol=1e-15)
    np.testing.assert_allclose(d, delta, rtol=0, atol=1e-15)
    assert _same_set(x, _expected_across(theta, delta, CUBE), 1e-14)
    # and no corner of either is inside the other, nor an edge-edge contact
    assert not any(_inside(c, pP, RP, hP) for c in _corners(pQ, RQ, hQ))
    assert not any(_inside(c, pQ, RQ, hQ) for c in _corners(pP, RP, hP))
    assert O.edge_contact(pP, RP, hP, pQ, RQ, hQ) is None


def test_rigid_motion_moves_the_contacts():
    rng = np.random.default_rng(4)
    pP, RP, hP, pQ, RQ, hQ = _across(np.radians(17.0), 3e-3)
    c, s_ = np.cos(0.004), np.sin(0.004)
    RQ = RQ @ np.array([[1, 0, 0], [0, c, -s_], [0, s_, c]])   # a small roll: the cube's z face least, clearly
    x0, d0, n0, w0 = O.face_contacts(pP, RP, hP, pQ, RQ, hQ)
    assert len(x0) == 4
    for _ in range(10):
        G, t = _random_rotation(rng), rng.normal(size=3)
        x, d, n, w = O.face_contacts(G @ pP + t, G @ RP, hP, G @ pQ + t, G @ RQ, hQ)
        assert w == w0 and len(x) == len(x0)
        np.testing.assert_allclose(n, G @ n0, atol=1e-13)
        np.testing.assert_allclose(d, d0, atol=1e-13)
        assert _same_set(x, x0 @ G.T + t, 1e-12)


def _sutherland_hodgman(poly, planes):
    """Clip a convex polygon (list of 2D points) by half-planes a . x <= b."""
    for a, b in planes:
        out = []
        for i in range(len(poly)):
            P, Q = poly[i], poly[(i + 1) % len(poly)]
            fp, fq = a @ P - b, a @ Q - b
            if fp <= 0:
                out.append(P)
            if (fp < 0 < fq) or (fq < 0 < fp):
                out.append(P + (Q - P) * (fp / (fp - fq)))
        poly = out
        if not poly:
            break
    return poly


def _brute_force(pP, RP, hP, pQ, RQ, hQ, n, who):
    """Reference face: the face of the other box facing the points' box with
    outward normal n; incident face: the points' box's face most anti-parallel
    to n; their 2D clip by Sutherland-Hodgman, lifted onto the incident face,
    kept below the reference face."""
    pI, RI, hI, pR, RR, hR = (pQ, RQ, hQ, pP, RP, hP) if who == "Q" else (pP, RP, hP, pQ, RQ, hQ)
    k = int(np.argmax(np.abs(RR.T @ n)))
    cR = pR + n * hR[k]
    r = [i for i in range(3) if i != k]
    A = RR[:, r]                                             # in-plane axes of the reference face
    j = int(np.argmax(np.abs(RI.T @ n)))
    sg = -1.0 if RI[:, j] @ n > 0 else 1.0
    cI = pI + RI[:, j] * sg * hI[j]
    i_ = [i for i in range(3) if i != j]
    B = RI[:, i_]
    quad = [cI + B @ np.array([sx * hI[i_[0]], sy * hI[i_[1]]]) for sx, sy in ((-1, -1), (1, -1), (1, 1), (-1, 1))]
    poly = [A.T @ (q - cR) for q in quad]
    e = hR[r]
    planes = [(np.array([1.0, 0]), e[0]), (np.array([-1.0, 0]), e[0]), (np.array([0, 1.0]), e[1]),
              (np.array([0, -1.0]), e[1])]
    clip = _sutherland_hodgman(poly, planes)
    M = A.T @ B                                              # incident-face coordinates -> plane coordinates
    off = A.T @ (cI - cR)
    pts = []
    for v in clip:
        uw = np.linalg.solve(M, v - off)
        x = cI + B @ uw
        if n @ (cR - x) > 0:
            pts.append(x)
    # remove duplicates of the polygon (vertices the clip repeats on a boundary)
    uniq = []
    for p in pts:
        if all(np.linalg.norm(p - q) > 1e-12 for q in uniq):
            uniq.append(p)
    return np.array(uniq).reshape(-1, 3)


def test_perturbed_crossings_against_sutherland_hodgman():
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(400):
        # a brick of random proportions across the cube's top face: turned about
        # the vertical, rolled about its length (its lowest edge stays level),
        # pitched by at most 1 mrad, its lowest point delta below the face
        hQ = np.array([rng.uniform(0.08, 0.3), rng.uniform(0.01, 0.04), rng.uniform(0.01, 0.04)])
        yaw, roll, pitch = rng.uniform(-0.7, 0.7), rng.uniform(-0.6, 0.6), rng.uniform(-1e-3, 1e-3)
        cr, sr, cp, sp = np.cos(roll), np.sin(roll), np.cos(pitch), np.sin(pitch)
        RQ = _rz(yaw) @ np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]]) @ np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
        low = np.abs(RQ[2]) @ hQ
        pQ = np.array([rng.uniform(-0.01, 0.01), rng.uniform(-0.01, 0.01), CUBE + low - rng.uniform(5e-4, 8e-3)])
        pP, RP, hP = np.zeros(3), np.eye(3), np.full(3, CUBE)
        G, t = _random_rotation(rng), rng.normal(size=3)
        pP, RP, pQ, RQ = G @ pP + t, G @ RP, G @ pQ + t, G @ RQ
        if rng.random() < 0.5:
            pP, RP, hP, pQ, RQ, hQ = pQ, RQ, hQ, pP, RP, hP
        if any(_inside(c, pP, RP, hP) for c in _corners(pQ, RQ, hQ)) or \
                any(_inside(c, pQ, RQ, hQ) for c in _corners(pP, RP, hP)):
            continue
        x, d, n, who = O.face_contacts(pP, RP, hP, pQ, RQ, hQ)
        if len(x) == 0:
            continue
        ref = _brute_force(pP, RP, hP, pQ, RQ, hQ, n, who)
        assert _same_set(x, ref, 1e-12)
        # depth: how far below the reference face, along n
        pR, RR, hR = (pP, RP, hP) if who == "Q" else (pQ, RQ, hQ)
        k = int(np.argmax(np.abs(RR.T @ n)))
        np.testing.assert_allclose(d, (pR + n * hR[k] - x) @ n, atol=1e-13)
        assert (d > 0).all() and len(x) <= 8
        checked += 1
    assert checked >= 200


def test_no_face_contact_when_apart_corner_inside_or_edge_axis():
    pP, RP, hP, pQ, RQ, hQ = _across(0.3, -1e-3)               # 1 mm apart
    assert len(O.face_contacts(pP, RP, hP, pQ, RQ, hQ)[0]) == 0
    # a small cube sunk into a big one's face: its corners are inside (corner contacts instead)
    I = np.eye(3)
    x, _, _, _ = O.face_contacts(np.zeros(3), I, [0.1] * 3, [0.0, 0.0, 0.1 + 0.02 - 0.005], I, [0.02] * 3)
    assert len(x) == 4                                           # the clip itself still finds the face
    # two crossing edges: the least overlap is an edge pair, no face contacts
    s2 = np.sqrt(2.0)
    Rx = np.array([[1, 0, 0], [0, 1 / s2, -1 / s2], [0, 1 / s2, 1 / s2]])
    Ry = np.array([[1 / s2, 0, 1 / s2], [0, 1, 0], [-1 / s2, 0, 1 / s2]])
    h = 0.05
    pQ = np.array([0.0, 0.0, -2 * h * s2 + 1e-3])
    assert O.edge_contact(np.zeros(3), Rx, [h] * 3, pQ, Ry, [h] * 3) is not None
    assert len(O.face_contacts(np.zeros(3), Rx, [h] * 3, pQ, Ry, [h] * 3)[0]) == 0


def test_edges_in_parallel_planes_stay_a_face_case():
    """The brick's long edges lie in planes parallel to the cube's face, so the
    cross products of the cube's x and y with the brick's length are the face
    normal with the same overlap: the face contacts win, under any rigid
    motion (where rounding would otherwise pick the edge pair)."""
    rng = np.random.default_rng(8)
    pP, RP, hP, pQ, RQ, hQ = _across(np.radians(12.0), 2e-3)
    for _ in range(20):
        G, t = _random_rotation(rng), rng.normal(size=3)
        args = (G @ pP + t, G @ RP, hP, G @ pQ + t, G @ RQ, hQ)
        assert O.edge_contact(*args) is None
        x, d, n, w = O.face_contacts(*args)
        assert len(x) == 4
        np.testing.assert_allclose(d, 2e-3, atol=1e-12)


def test_robot_detect_lists_the_face_contacts():
    """In the oracle's contact detection (twisted robots), a pair with no
    corner inside and no edge-edge contact gets exactly face_contacts of its
    two boxes, in order, on the incident box (corner code -4)."""
    found = 0
    for key in range(30, 60):
        pop = dataclasses.replace(W.twisted_chains(8, nh=6, key=key), self_collision=True)
        o = O.Oracle(pop, float32_constants=False)
        for step in range(0, 400, 20):
            for vi in range(pop.n_variants):
                q = o.variant_state(vi)[0]
                c = o.contacts(vi, q, max_contacts=4096)
                sel = np.where(c["corner"] == -4)[0]
                if not len(sel):
                    continue
                R, p, _, _ = o.fk(vi, q)
                b0 = pop.body_offset[vi]
                half = pop.half_ext[b0:b0 + R.shape[0]].astype(np.float64)
                pairs = sorted({(min(int(c["body"][k]), int(c["other"][k])),
                                 max(int(c["body"][k]), int(c["other"][k]))) for k in sel})
                for a, b in pairs:
                    ks = [k for k in sel if {int(c["body"][k]), int(c["other"][k])} == {a, b}]
                    x, d, n, who = O.face_contacts(p[a], R[a], half[a], p[b], R[b], half[b])
                    assert len(x) == len(ks)
                    owner = b if who == "Q" else a
                    for i, k in enumerate(ks):
                        assert int(c["body"][k]) == owner
                        np.testing.assert_allclose(c["x"][k], x[i], atol=1e-12)
                        np.testing.assert_allclose(c["depth"][k], d[i], atol=1e-12)
                    found += 1
            o.step(20)
            if found >= 5:
                return
    assert found >= 5
