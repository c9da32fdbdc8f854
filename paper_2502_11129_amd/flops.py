"""Algorithmic work of one simulation step (for roofline reporting).

Flops of the dense method per variant-step, at each variant's own sizes
(nh hinges, nb bodies, nv DoFs, D = sum of body depths) and its actually
active rows (n_c contacts, n_clamp engaged actuator clamps), FMA = 2:

  156 nh + 594 nb + 60 D + 72 nh          kinematics, RNEA, CRBA, control
  + (2/3) nv^3 + 2 nv^2 + 100             dense factorisation and free solve
  + n_c (50 + 9 dbar + 6 nv^2 + 6 nv + 12 K nv)   contact rows and K sweeps
  + n_clamp (2 nv^2 + 4 K nv)             clamp rows and K sweeps
  + 70 nb + 60                            with a ball: ball-box tests, ball update
  + 12 nb (nb - 1) / 2                    with self-collision: bounding-sphere tests

(nv counts the ball's six DoFs when there is one.)  With the tree-sparse
factorisation (`factorization` "tree" for a variant) the factorisation and
every solve are counted at the sparse algorithm's flops instead
(`factor_solve_flops`): (2/3) nv^3 + 2 nv^2 becomes factor + solve, the
contact rows' 6 nv^2 three solves and a clamp row's 2 nv^2 one solve.

Padded lanes, bin capacities and the kernel's own extra work (for instance
the explicit inverse) are not counted.  Bytes: model + state read once and
state + fitness written once per rollout launch.
"""
from __future__ import annotations

import numpy as np


def depth_sums(pop):
    """Sum of body depths and mean depth per variant."""
    D = np.zeros(pop.n_variants)
    dbar = np.zeros(pop.n_variants)
    bo = pop.body_offset
    for i in range(pop.n_variants):
        par = pop.parent[bo[i]:bo[i + 1]]
        d = np.zeros(len(par))
        for b in range(1, len(par)):
            d[b] = d[par[b]] + 1
        D[i] = d.sum()
        dbar[i] = d.mean()
    return D, dbar


def flops_per_variant(pop, steps, rows_contact, rows_clamp, K=None, factorization="dense"):
    """Algorithmic flops of `steps` steps per variant given the counters
    (rows_contact = sum of active contacts over those steps, rows_clamp = sum
    of engaged clamps); factorization: "dense", "tree" or one of them per
    variant."""
    K = int(pop.params["pgs_iters"] if K is None else K)
    nh = pop.n_hinges.astype(np.float64)
    nb = pop.n_bodies.astype(np.float64)
    nv = pop.nv.astype(np.float64)
    D, dbar = depth_sums(pop)
    fac = np.broadcast_to(np.asarray(factorization), (pop.n_variants,))
    factor, solve = (2.0 / 3.0) * nv ** 3, 2 * nv ** 2
    if (fac == "tree").any():
        tf, ts = factor_solve_flops(pop, "tree")
        factor = np.where(fac == "tree", tf, factor)
        solve = np.where(fac == "tree", ts, solve)
    base = 156 * nh + 594 * nb + 60 * D + 72 * nh + factor + solve + 100
    if getattr(pop, "ball", None) is not None:
        base = base + 70 * nb + 60
    if getattr(pop, "self_collision", False):
        base = base + 12 * nb * (nb - 1) / 2        # bounding-sphere tests of every body pair
    per_contact = 50 + 9 * dbar + 3 * solve + 6 * nv + 12 * K * nv
    per_clamp = solve + 4 * K * nv
    return (base * steps + np.asarray(rows_contact, np.float64) * per_contact
            + np.asarray(rows_clamp, np.float64) * per_clamp)


def dof_parents(pop, i):
    """Parent of every DoF of variant i in the DoF tree of the tree-sparse
    factorisation (-1 at a root): a free root's six DoFs form a chain, a
    hinge hangs under the hinge of its body's parent (under the root's last
    DoF for a child of the core), a ball's six DoFs are roots of their own."""
    bo = pop.body_offset
    par = pop.parent[bo[i]:bo[i + 1]]
    ball = getattr(pop, "ball", None) is not None
    r0 = int(pop.nv[i]) - (len(par) - 1) - (6 if ball else 0)
    lam = list(range(-1, r0 - 1))
    for b in range(1, len(par)):
        lam.append(r0 - 1 if par[b] == 0 else r0 + int(par[b]) - 1)
    return np.asarray(lam + ([-1] * 6 if ball else []), np.int64)


def factor_solve_flops(pop, kind):
    """Per variant: (flops of one factorisation, flops of one solve) of the
    joint-space system in the host worker, FMA = 2: "dense" Cholesky
    (nv^3 / 3, 2 nv^2) or "tree"-sparse L^T L, where DoF k with ancestors
    anc(k) costs a square root, |anc(k)| divisions and, per ancestor i,
    |anc(i)| + 1 multiply-adds, and a solve two sweeps of |anc(k)|
    multiply-adds plus a division per DoF."""
    nv = pop.nv.astype(np.float64)
    if kind == "dense":
        return nv ** 3 / 3.0, 2.0 * nv ** 2
    fac = np.zeros(pop.n_variants)
    sol = np.zeros(pop.n_variants)
    for v in range(pop.n_variants):
        lam = dof_parents(pop, v)
        na = np.zeros(len(lam), np.int64)          # ancestors per DoF (parents come first)
        for k in range(len(lam)):
            na[k] = 0 if lam[k] < 0 else na[lam[k]] + 1
        f = 0.0
        for k in range(len(lam)):
            f += 1 + na[k]
            j = lam[k]
            while j >= 0:
                f += 2.0 * (na[j] + 1)
                j = lam[j]
        fac[v] = f
        sol[v] = 4.0 * na.sum() + 2.0 * len(lam)
    return fac, sol


def bytes_per_rollout(pop):
    """Algorithmic HBM bytes of one rollout launch: model (24 words per body,
    header) and initial state read, final state and fitness written."""
    nb = pop.n_bodies.astype(np.float64)
    nq = pop.nq.astype(np.float64)
    nv = pop.nv.astype(np.float64)
    return float((4 * (24 * nb + 16) + 4 * (nq + nv) * 2 + 4 + 16).sum())
