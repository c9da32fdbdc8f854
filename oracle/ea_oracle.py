"""Reference of the evolutionary outer loop's variation and selection steps
(TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the product path never
loads it).

The paper motivates the work by evolutionary robotics with Revolve2, a
memetic (Lamarckian) evolution of body and controller (Sec. 1); it fixes no
operator.  The operators below are this build's reading, written plainly
over numpy arrays of the genotype layout (hinge j joins body j+1 to
parent[j] on face[j] with axis flag axis[j]; cpg[j] = (A, omega, phi);
padding -1 / 0):

* random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
  Random Numbers: As Easy as 1, 2, 3", SC 2011), key = the 64-bit seed,
  counter = (offspring, generation, block, row); a uniform is
  (x >> 8) * 2^-24 and an index below n is the high half of x * n;
* parent choice: two binary tournaments (the higher fitness wins, NaN loses,
  ties go to the lower index);
* crossover: the first parent's body; each of its CPG rows j is taken from
  the second parent when bit j of a random word is set and j < nh2;
* body mutation (probability 0.3): one of add a leaf brick (uniform over
  the free slots of bodies of depth < 4, as the random-tree generator
  enumerates them), remove a leaf brick (uniform over childless bricks, later
  bodies renumbered), flip one hinge's axis; impossible operations (20 or 4
  hinges) change nothing;
* CPG mutation: each row with probability 0.2 moves A by 0.1 t, omega by
  0.5 t, phi by 0.5 t with t uniform in [-1, 1) (one draw each), A clamped to
  [0, 1], omega to [1, 6], phi wrapped into [0, 2 pi); all in float32;
* Lamarckian tuning: every row moves by (0.05, 0.25, 0.25) t, the same
  clamps; a tuned controller replaces the base one when its fitness is
  strictly higher;
* survivors: the mu best of parents then offspring (ties to the lower
  position, NaN last).
"""
from __future__ import annotations

import numpy as np

MAXH = 20
P_MORPH = np.float32(0.3)
P_CPG = np.float32(0.2)
SIG_VARY = (np.float32(0.1), np.float32(0.5), np.float32(0.5))
SIG_TUNE = (np.float32(0.05), np.float32(0.25), np.float32(0.25))
TWO_PI = np.float32(2.0 * np.pi)
# allowed faces per body: the core uses +x, -x, +y, -y (codes 0..3), bricks +x, +y, -y
CORE_FACES = (0, 1, 2, 3)
BRICK_FACES = (0, 2, 3)
MAX_DEPTH = 4


def philox4x32(ctr, key, rounds=10):
    """Philox4x32-10 of one 128-bit counter and 64-bit key (Python ints)."""
    c0, c1, c2, c3 = (int(x) & 0xFFFFFFFF for x in ctr)
    k0, k1 = (int(x) & 0xFFFFFFFF for x in key)
    for r in range(rounds):
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF, \
                         ((p0 >> 32) ^ c3 ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF
        if r < rounds - 1:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
    return c0, c1, c2, c3


def draws(seed, i, g, block, row=0):
    return philox4x32((i, g, block, row), (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))


def unif(x):
    """float32 uniform in [0, 1) from the top 24 bits."""
    return np.float32((x >> 8) * 2.0 ** -24)


def below(x, n):
    """Index in [0, n) from a 32-bit word: high half of x * n."""
    return (int(x) * int(n)) >> 32


def _better(f, a, b):
    fa, fb = f[a], f[b]
    if np.isnan(fa):
        return b if not np.isnan(fb) else min(a, b)
    if np.isnan(fb):
        return a
    if fa > fb:
        return a
    if fb > fa:
        return b
    return min(a, b)


def _depths(parent, nh):
    d = [0] * (nh + 1)
    for j in range(nh):
        d[j + 1] = d[parent[j]] + 1
    return d


def free_slots(parent, face, nh):
    """Free (body, face) slots in body order, faces in code order."""
    used = set((int(parent[j]), int(face[j])) for j in range(nh))
    depth = _depths(parent, nh)
    out = []
    for b in range(nh + 1):
        if depth[b] >= MAX_DEPTH:
            continue
        for f in (CORE_FACES if b == 0 else BRICK_FACES):
            if (b, f) not in used:
                out.append((b, f))
    return out


def leaves(parent, nh):
    """Childless bricks (body indices 1..nh) in body order."""
    has_child = set(int(parent[j]) for j in range(nh))
    return [b for b in range(1, nh + 1) if b not in has_child]


def _move(v, t, sig, lo, hi):
    return np.float32(min(hi, max(lo, np.float32(v + np.float32(sig * t)))))


def _wrap(v, t, sig):
    p = np.float32(v + np.float32(sig * t))
    if p < 0:
        p = np.float32(p + TWO_PI)
    elif p >= TWO_PI:
        p = np.float32(p - TWO_PI)
    return p


def _signed(x):
    """t = 2 u - 1 in [-1, 1) (exact in float32)."""
    return np.float32(np.float32(2.0) * unif(x) - np.float32(1.0))


def perturb_row(row, xs, sig):
    A, om, ph = (np.float32(v) for v in row)
    return (_move(A, _signed(xs[0]), sig[0], np.float32(0), np.float32(1)),
            _move(om, _signed(xs[1]), sig[1], np.float32(1), np.float32(6)),
            _wrap(ph, _signed(xs[2]), sig[2]))


def add_leaf(nh, parent, face, axis, cpg, word, flag, row):
    """New brick on free slot below(word, #slots) (in place); returns nh."""
    if nh >= MAXH:
        return nh
    slots = free_slots(parent, face, nh)
    if not slots:
        return nh
    b, f = slots[below(word, len(slots))]
    parent[nh], face[nh], axis[nh] = b, f, int(flag)
    cpg[nh] = row
    return nh + 1


def remove_leaf(nh, parent, face, axis, cpg, word):
    """Remove childless brick below(word, #leaves) and renumber the later
    bodies (in place); returns nh."""
    if nh <= 4:
        return nh
    lv = leaves(parent, nh)
    L = lv[below(word, len(lv))]          # body L, joined by hinge L - 1
    for j in range(L - 1, nh - 1):
        parent[j], face[j], axis[j] = parent[j + 1], face[j + 1], axis[j + 1]
        cpg[j] = cpg[j + 1]
    for j in range(nh - 1):
        if parent[j] > L:
            parent[j] -= 1
    nh -= 1
    parent[nh] = face[nh] = axis[nh] = -1
    cpg[nh] = 0
    return nh


def flip_axis(nh, axis, word):
    j = below(word, nh)
    axis[j] ^= 1


def vary_one(i, g, seed, nh_p, parent_p, face_p, axis_p, cpg_p, fit):
    """Offspring i of generation g: returns (nh, parent[20], face[20], axis[20], cpg[20,3])."""
    mu = len(nh_p)
    x = draws(seed, i, g, 0)
    p1 = _better(fit, below(x[0], mu), below(x[1], mu))
    p2 = _better(fit, below(x[2], mu), below(x[3], mu))
    nh = int(nh_p[p1])
    parent = [int(v) for v in parent_p[p1]]
    face = [int(v) for v in face_p[p1]]
    axis = [int(v) for v in axis_p[p1]]
    cpg = np.array(cpg_p[p1], dtype=np.float32).copy()
    # crossover of controller rows
    xc = draws(seed, i, g, 1)
    nh2 = int(nh_p[p2])
    for j in range(nh):
        if (xc[0] >> j) & 1 and j < nh2:
            cpg[j] = cpg_p[p2][j]
    # body mutation
    if unif(xc[1]) < P_MORPH:
        op = below(xc[2], 3)
        if op == 0:
            xn = draws(seed, i, g, 2)
            row = (unif(xn[0]), np.float32(np.float32(1) + np.float32(np.float32(5) * unif(xn[1]))),
                   np.float32(TWO_PI * unif(xn[2])))
            nh = add_leaf(nh, parent, face, axis, cpg, xc[3], xn[3] & 1, row)
        elif op == 1:
            nh = remove_leaf(nh, parent, face, axis, cpg, xc[3])
        else:
            flip_axis(nh, axis, xc[3])
    # controller mutation
    for j in range(nh):
        xr = draws(seed, i, g, 3, j)
        if unif(xr[0]) < P_CPG:
            cpg[j] = perturb_row(cpg[j], xr[1:], SIG_VARY)
    for j in range(nh, MAXH):
        parent[j] = face[j] = axis[j] = -1
        cpg[j] = 0
    return nh, parent, face, axis, cpg


def vary(g, seed, parents, fit, n_off):
    """Offspring arrays (dict of nh, parent, face, axis, cpg) of generation g."""
    nh = np.zeros(n_off, np.int32)
    par = -np.ones((n_off, MAXH), np.int32)
    fac = -np.ones((n_off, MAXH), np.int32)
    axs = -np.ones((n_off, MAXH), np.int32)
    cpg = np.zeros((n_off, MAXH, 3), np.float32)
    for i in range(n_off):
        r = vary_one(i, g, seed, parents["nh"], parents["parent"], parents["face"], parents["axis"],
                     parents["cpg"], np.asarray(fit, np.float32))
        nh[i], par[i], fac[i], axs[i], cpg[i] = r[0], r[1], r[2], r[3], r[4]
    return dict(nh=nh, parent=par, face=fac, axis=axs, cpg=cpg)


def tune_perturb(g, seed, round_, base):
    """Lamarckian candidate controllers: every row of every genotype moved."""
    out = {k: v.copy() for k, v in base.items()}
    n = len(base["nh"])
    for i in range(n):
        for j in range(int(base["nh"][i])):
            xr = draws(seed, i, g, 64 + round_, j)
            out["cpg"][i, j] = perturb_row(base["cpg"][i, j], xr[:3], SIG_TUNE)
    return out


def tune_accept(base, fbase, cand, fcand):
    """Keep a candidate controller whose fitness is strictly higher."""
    cpg = base["cpg"].copy()
    f = np.asarray(fbase, np.float32).copy()
    for i in range(len(f)):
        if fcand[i] > f[i] or (np.isnan(f[i]) and not np.isnan(fcand[i])):
            cpg[i] = cand["cpg"][i]
            f[i] = fcand[i]
    out = {k: v.copy() for k, v in base.items()}
    out["cpg"] = cpg
    return out, f


def survivors(fit_parents, fit_off, mu):
    """Positions (parents first, then offspring) of the mu best, ascending."""
    f = np.concatenate([np.asarray(fit_parents, np.float64), np.asarray(fit_off, np.float64)])
    key = np.where(np.isnan(f), -np.inf, f)
    order = sorted(range(len(f)), key=lambda k: (-key[k], np.isnan(f[k]), k))
    return np.array(sorted(order[:mu]), np.int64)
