"""Pins of the oracle's self-collision (corners of a box inside another box of
the same robot not joined to it by a hinge, one separating-axis normal per
pair) against an independent brute-force enumeration over the oracle's own
forward kinematics (point-in-box tests and a separating-axis search written
here; an edge-edge contact only for pairs with no corner inside, with the
depth of the boxes' corner supports along its normal), rigid-motion
invariance of the rows, a folding chain that passes
through itself without the contacts and stops with them, and quadrupeds
whose limbs meet without the solver failing."""
import dataclasses

import numpy as np

from oracle import oracle as O
from paper_2502_11129_amd import workloads as W


def _corners(p, R, h):
    s = np.array([[(1 if c & 1 else -1) * h[0], (1 if c & 2 else -1) * h[1], (1 if c & 4 else -1) * h[2]]
                  for c in range(8)])
    return p + s @ R.T


def _sat_axis(pP, RP, hP, pQ, RQ, hQ):
    """Least-overlap separating axis (P faces, Q faces, edge crosses), from Q to P."""
    d = pP - pQ
    axes = [RP[:, k] for k in range(3)] + [RQ[:, k] for k in range(3)]
    for i in range(3):
        for j in range(3):
            c = np.cross(RP[:, i], RQ[:, j])
            if c @ c >= 1e-6:
                axes.append(c / np.linalg.norm(c))
    over = [hP @ np.abs(RP.T @ u) + hQ @ np.abs(RQ.T @ u) - abs(u @ d) for u in axes]
    u = axes[int(np.argmin(over))]
    return u if u @ d >= 0 else -u


def _brute_force(o, pop, vi, q, band=0.0):
    """(body, other, corner, depth, normal, x) of every corner strictly inside
    a non-adjacent box, in the order pairs (a < b), corners of a then of b,
    with the pair's separating-axis normal and the corner's depth along it;
    with band > 0, also the set of corners within `band` of a box surface
    (where rounding decides)."""
    R, p, _, _ = o.fk(vi, q)
    b0 = pop.body_offset[vi]
    nb = R.shape[0]
    par = pop.parent[b0:b0 + nb]
    half = pop.half_ext[b0:b0 + nb].astype(np.float64)
    out, ambiguous = [], set()
    for a in range(nb):
        for b in range(a + 1, nb):
            if par[b] == a:
                continue
            hits = []
            for P, Q in ((a, b), (b, a)):
                for c, x in enumerate(_corners(p[P], R[P], half[P])):
                    l = R[Q].T @ (x - p[Q])
                    if (np.abs(np.abs(l) - half[Q]) <= band).any() and (np.abs(l) <= half[Q] + band).all():
                        ambiguous.add((P, Q, c))
                        continue
                    if (np.abs(l) < half[Q]).all():
                        hits.append((P, Q, c, x))
            if not hits:
                continue
            u = _sat_axis(p[a], R[a], half[a], p[b], R[b], half[b])
            for P, Q, c, x in hits:
                n = u if P == a else -u
                depth = n @ p[Q] + half[Q] @ np.abs(R[Q].T @ n) - n @ x
                out.append((P, Q, c, depth, n, x))
    return (out, ambiguous) if band > 0 else out


def _twisted_trees(n=12, seed=3):
    pop = W.random_trees(n)
    pop = dataclasses.replace(pop, self_collision=True)
    rng = np.random.default_rng(seed)
    q0 = pop.q0.copy()
    for i in range(n):
        qo = pop.q_offset[i]
        nh = int(pop.n_hinges[i])
        q0[qo + 7:qo + 7 + nh] = rng.uniform(-2.6, 2.6, nh)
    return dataclasses.replace(pop, q0=q0)


def test_self_contacts_against_brute_force_enumeration():
    pop = _twisted_trees()
    o = O.Oracle(pop, float32_constants=False)
    total = 0
    for vi in range(pop.n_variants):
        q = o.variant_state(vi)[0]
        c = o.contacts(vi, q, max_contacts=4096)
        want, ambiguous = _brute_force(o, pop, vi, q, band=1e-12)
        # corners within rounding of a box surface may go either way
        sel = [k for k in np.where((c["other"] >= 0) & (c["corner"] >= 0))[0]
               if (int(c["body"][k]), int(c["other"][k]), int(c["corner"][k])) not in ambiguous]
        assert len(sel) == len(want)
        # edge-edge contacts (corner -3) only for pairs with no corner inside or near a
        # surface, with the depth the overlap of the two boxes' corner supports along n
        R, p, _, _ = o.fk(vi, q)
        b0 = pop.body_offset[vi]
        half = pop.half_ext[b0:b0 + R.shape[0]].astype(np.float64)
        near = {(P, Q) for P, Q, _ in ambiguous} | {(P, Q) for P, Q, *_ in want}
        for k in np.where(c["corner"] == -3)[0]:
            P, Q = int(c["body"][k]), int(c["other"][k])
            assert (P, Q) not in near and (Q, P) not in near
            n = c["normal"][k]
            ov = (_corners(p[Q], R[Q], half[Q]) @ n).max() - (_corners(p[P], R[P], half[P]) @ n).min()
            np.testing.assert_allclose(c["depth"][k], ov, rtol=0, atol=1e-12)
        for k, (P, Q, corner, depth, n, x) in zip(sel, want):
            assert (c["body"][k], c["other"][k], c["corner"][k]) == (P, Q, corner)
            np.testing.assert_allclose(c["depth"][k], depth, rtol=0, atol=1e-12)
            np.testing.assert_allclose(c["normal"][k], n, rtol=0, atol=1e-12)
            np.testing.assert_allclose(c["x"][k], x, rtol=0, atol=1e-13)
        total += len(sel)
    assert total > 20


def test_self_contact_rows_vanish_for_rigid_motion_of_the_robot():
    """Internal contacts: moving the whole robot rigidly (root velocities
    only) moves both boxes' points alike, so every self-contact row is zero."""
    pop = _twisted_trees(8, seed=4)
    o = O.Oracle(pop, float32_constants=False)
    rng = np.random.default_rng(1)
    seen = 0
    for vi in range(pop.n_variants):
        q = o.variant_state(vi)[0]
        c = o.contacts(vi, q, max_contacts=4096)
        sel = c["other"] >= 0
        if not sel.any():
            continue
        v = np.zeros(c["J"].shape[2])
        v[:6] = rng.normal(size=6)
        assert np.abs(c["J"][sel] @ v).max() < 1e-13
        # and the normal row of a contact separates the two boxes: moving the
        # corner's box along +n with the other fixed gives +1 per unit speed
        seen += int(sel.sum())
    assert seen > 10


def _max_self_penetration(o, pop, q):
    """Deepest corner of one box inside another (distance to the nearest face)."""
    R, p, _, _ = o.fk(0, q)
    half = pop.half_ext[:R.shape[0]].astype(np.float64)
    worst = 0.0
    for P, Q, c, _, _, x in _brute_force(o, pop, 0, q):
        l = R[Q].T @ (x - p[Q])
        worst = max(worst, float((half[Q] - np.abs(l)).min()))
    return worst


def test_folding_chain_passes_through_itself_without_contacts_and_stops_with_them():
    prm = dict(W.DEFAULT_PARAMS)
    prm["gravity"] = (0.0, 0.0, 0.0)
    worst = {}
    for sc in (False, True):
        pop = W.chain(4, ["+x"] * 4, [0] * 4, root_type=W.ROOT_FIXED, cpg=[(1.0, 2.0, 1.57)] * 4, params=prm)
        pop = dataclasses.replace(pop, self_collision=sc)
        o = O.Oracle(pop, float32_constants=False)
        w = 0.0
        for _ in range(150):
            o.step(10)
            w = max(w, _max_self_penetration(o, pop, o.variant_state(0)[0]))
        worst[sc] = w
    assert worst[False] > 0.015         # the tip sweeps through the core
    assert worst[True] < 0.005          # held at the soft contact's millimetre scale


def test_quadruped_limbs_meet_without_solver_failure():
    """Limbs swinging on vertical hinges meet side by side at equal height: a
    nearest-face normal there would be vertical, where no joint can push; the
    separating-axis normal is horizontal and the run stays finite."""
    pop = dataclasses.replace(W.quadrupeds(64), self_collision=True)
    o = O.Oracle(pop, float32_constants=False)
    o.step(1000, 8)
    a, _ = o.counters()
    o0 = O.Oracle(W.quadrupeds(64), float32_constants=False)
    o0.step(1000, 8)
    a0, _ = o0.counters()
    assert (o.get_state()[3] == 0).all()
    assert ((a.astype(np.int64) - a0.astype(np.int64)) > 0).sum() >= 10   # self-contacts happened


def _fibonacci_sphere(n):
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(1.0 - z * z)
    a = np.pi * (3.0 - np.sqrt(5.0)) * i
    return np.stack([r * np.cos(a), r * np.sin(a), z], axis=1)


def test_self_contact_normal_is_the_least_overlap_direction_over_all_directions():
    """Independent of the separating-axis enumeration: for every box pair with
    a corner contact, the translation along the oracle's normal that
    separates the boxes (largest projection of the other box's corners minus
    the smallest of the corner box's) is no larger than along any of 400 000
    directions spread over the sphere, and within the grid's resolution of
    the smallest of them (the least translation, the penetration depth of
    the pair); the normal points from the other box to the corner box; each
    corner's depth is the other box's largest corner projection along the
    normal minus the corner's own."""
    pop = _twisted_trees(10, seed=5)
    o = O.Oracle(pop, float32_constants=False)
    U = _fibonacci_sphere(400_000)
    seen = 0
    for vi in range(pop.n_variants):
        q = o.variant_state(vi)[0]
        c = o.contacts(vi, q, max_contacts=4096)
        R, p, _, _ = o.fk(vi, q)
        b0 = pop.body_offset[vi]
        half = pop.half_ext[b0:b0 + R.shape[0]].astype(np.float64)
        done = set()
        for k in np.where((c["other"] >= 0) & (c["corner"] >= 0))[0]:
            P, Q = int(c["body"][k]), int(c["other"][k])
            n = np.asarray(c["normal"][k], np.float64)
            cP, cQ = _corners(p[P], R[P], half[P]), _corners(p[Q], R[Q], half[Q])
            assert abs(np.linalg.norm(n) - 1.0) < 1e-6      # rotations of the float32 state quaternion
            assert n @ (p[P] - p[Q]) >= -1e-12
            np.testing.assert_allclose(c["depth"][k], (cQ @ n).max() - c["x"][k] @ n, rtol=0, atol=1e-12)
            if (min(P, Q), max(P, Q)) in done:
                continue
            done.add((min(P, Q), max(P, Q)))
            ov_n = (cQ @ n).max() - (cP @ n).min()
            proj_P, proj_Q = cP @ U.T, cQ @ U.T
            # the translation along u that separates the boxes (P moved ahead of Q)
            ov = proj_Q.max(0) - proj_P.min(0)
            assert ov_n <= ov.min() + 1e-9
            assert ov_n >= ov.min() - 2e-3 * np.linalg.norm(half[P] + half[Q])
            seen += 1
    assert seen >= 10
