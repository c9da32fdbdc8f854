"""Pins of the evolutionary loop's reference operators (oracle/ea_oracle.py)
against things other than themselves: the published Philox4x32-10 known
answers, hand-worked tree edits, brute-force enumeration, exact
distributions, and structural validity of every offspring."""
import numpy as np
import pytest

from oracle import ea_oracle as E
from paper_2502_11129_amd import workloads as W


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 (Salmon et al., SC 2011)."""
    assert E.philox4x32((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert E.philox4x32((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert E.philox4x32((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_uniform_and_index_ranges():
    assert E.unif(0) == 0.0 and E.unif(0xFFFFFFFF) == np.float32(1 - 2 ** -24)
    for n in (1, 3, 7, 20, 4096, 100003):
        assert E.below(0, n) == 0 and E.below(0xFFFFFFFF, n) == n - 1
    # below() splits the 32-bit range into n nearly equal intervals
    counts = np.bincount([E.below(x, 3) for x in range(0, 1 << 32, 1 << 20)], minlength=3)
    assert counts.max() - counts.min() <= 1
    assert E._signed(0) == -1.0 and E._signed(0xFFFFFFFF) == np.float32(1 - 2 ** -23)


def _tree(edges):
    """Genotype lists of a hand-built tree: edges = [(parent, face, axis), ...]."""
    nh = len(edges)
    parent = [e[0] for e in edges] + [-1] * (20 - nh)
    face = [e[1] for e in edges] + [-1] * (20 - nh)
    axis = [e[2] for e in edges] + [-1] * (20 - nh)
    cpg = np.zeros((20, 3), np.float32)
    for j in range(nh):
        cpg[j] = (0.1 * (j + 1), 1.0 + j, 0.5 * j)
    return nh, parent, face, axis, cpg


def test_free_slots_and_leaves_worked_example():
    # core with bricks on +x (body 1) and +y (body 2); body 3 on body 1's +x; body 4 on body 3's -y
    nh, parent, face, axis, cpg = _tree([(0, 0, 0), (0, 2, 1), (1, 0, 0), (3, 3, 1)])
    # depths: 0, 1, 1, 2, 3 -> every body may still take children
    assert E.free_slots(parent, face, nh) == [(0, 1), (0, 3), (1, 2), (1, 3), (2, 0), (2, 2), (2, 3),
                                              (3, 0), (3, 2), (4, 0), (4, 2), (4, 3)]
    assert E.leaves(parent, nh) == [2, 4]
    # a brick at depth 4 takes no children
    nh, parent, face, axis, cpg = _tree([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0)])
    assert all(b != 4 for b, _ in E.free_slots(parent, face, nh))


def test_remove_leaf_worked_example():
    nh, parent, face, axis, cpg = _tree([(0, 0, 0), (0, 2, 1), (1, 0, 0), (3, 3, 1), (2, 2, 0)])
    # leaves: bodies 4 (on 3) and 5 (on 2); word 0 picks the first leaf, body 4 (hinge 3)
    nh2 = E.remove_leaf(nh, parent, face, axis, cpg, 0)
    assert nh2 == 4
    # hinge 4 (body 5 on body 2) moves to hinge 3; its parent 2 is below the removed body: unchanged
    assert parent[:5] == [0, 0, 1, 2, -1] and face[:5] == [0, 2, 0, 2, -1] and axis[:5] == [0, 1, 0, 0, -1]
    np.testing.assert_array_equal(cpg[3], np.float32([0.5, 5.0, 2.0]))
    assert (cpg[4] == 0).all()
    # removing body 2 (hinge 1) renumbers bodies 3.. down by one, parents too
    nh, parent, face, axis, cpg = _tree([(0, 0, 0), (0, 2, 1), (1, 0, 0), (3, 3, 1), (0, 3, 0)])
    assert E.leaves(parent, nh) == [2, 4, 5]
    nh2 = E.remove_leaf(nh, parent, face, axis, cpg, 0)
    assert parent[:4] == [0, 1, 2, 0] and face[:4] == [0, 0, 3, 3]


def test_remove_and_add_respect_size_limits():
    nh, parent, face, axis, cpg = _tree([(0, 0, 0), (0, 1, 0), (0, 2, 0), (0, 3, 0)])
    assert E.remove_leaf(nh, parent, face, axis, cpg, 12345) == 4
    g = W.random_genotypes(200, key=9)
    full = [i for i in range(200) if g.nh[i] == 20]
    assert full
    i = full[0]
    p, f, a, c = list(g.parent[i]), list(g.face[i]), list(g.axis[i]), g.cpg[i].copy()
    assert E.add_leaf(20, p, f, a, c, 77, 1, (0.5, 2.0, 1.0)) == 20


def _canonical(parent, face, nh):
    """Set of root paths (face sequences) of the bricks: a labelling-free form."""
    paths = {0: ()}
    for j in range(nh):
        paths[j + 1] = paths[parent[j]] + (face[j],)
    return sorted(paths[b] for b in range(1, nh + 1))


def test_remove_leaf_removes_exactly_one_path_brute_force():
    g = W.random_genotypes(300, key=3)
    for i in range(300):
        nh = int(g.nh[i])
        before = _canonical(g.parent[i], g.face[i], nh)
        for w in (0, 0x55555555, 0xFFFFFFFF):
            p, f, a, c = list(g.parent[i]), list(g.face[i]), list(g.axis[i]), g.cpg[i].copy()
            nh2 = E.remove_leaf(nh, p, f, a, c, w)
            after = _canonical(p, f, nh2)
            if nh == 4:
                assert after == before
                continue
            assert nh2 == nh - 1
            diff = list(before)
            for path in after:
                diff.remove(path)
            assert len(diff) == 1 and all(path[:len(diff[0])] != diff[0] for path in after)


def _valid(nh, parent, face, axis, cpg):
    assert 4 <= nh <= 20
    depth = [0]
    used = set()
    for j in range(nh):
        b = parent[j]
        assert 0 <= b <= j
        assert face[j] in ((0, 1, 2, 3) if b == 0 else (0, 2, 3))
        assert (b, face[j]) not in used
        used.add((b, face[j]))
        depth.append(depth[b] + 1)
        assert depth[-1] <= 4
        assert axis[j] in (0, 1)
        A, om, ph = cpg[j]
        assert 0.0 <= A <= 1.0 and 1.0 <= om <= 6.0 and 0.0 <= ph < np.float32(2 * np.pi)
    for j in range(nh, 20):
        assert parent[j] == face[j] == axis[j] == -1 and (cpg[j] == 0).all()


def _parents(mu, key=1):
    g = W.random_genotypes(mu, key=key)
    return dict(nh=g.nh, parent=g.parent, face=g.face, axis=g.axis, cpg=g.cpg)


def test_offspring_are_valid_trees():
    par = _parents(64)
    fit = np.random.default_rng(0).random(64).astype(np.float32)
    off = E.vary(3, 0xC0FFEE, par, fit, 600)
    for i in range(600):
        _valid(off["nh"][i], off["parent"][i], off["face"][i], off["axis"][i], off["cpg"][i])
    # every kind of change occurs
    nh_changes = set(np.sign(off["nh"].astype(int) - 0))
    assert len(set(off["nh"])) > 5


def test_binary_tournament_rank_distribution():
    """With distinct fitnesses, the first parent's fitness rank r (0 = worst)
    of a binary tournament over uniform draws has probability (2r + 1)/mu^2.
    Offspring whose body is unchanged identify their first parent."""
    mu = 16
    par = _parents(mu, key=5)
    fit = np.arange(mu, dtype=np.float32)          # rank = index
    n = 4000
    off = E.vary(0, 99, par, fit, n)
    keys = {tuple(par["parent"][k]) + tuple(par["face"][k]) + tuple(par["axis"][k]): k for k in range(mu)}
    assert len(keys) == mu
    ranks = []
    for i in range(n):
        k = keys.get(tuple(off["parent"][i]) + tuple(off["face"][i]) + tuple(off["axis"][i]))
        if k is not None:
            ranks.append(k)
    ranks = np.bincount(ranks, minlength=mu)
    expect = (2 * np.arange(mu) + 1) / mu ** 2 * ranks.sum()
    chi2 = ((ranks - expect) ** 2 / expect).sum()
    assert chi2 < 40.0, (chi2, ranks)                # 15 dof: p ~ 5e-4
    assert ranks.sum() > 0.6 * n


def test_nan_fitness_never_wins_a_tournament():
    mu = 8
    par = _parents(mu, key=6)
    fit = np.full(mu, np.nan, np.float32)
    fit[5] = -3.0
    off = E.vary(1, 7, par, fit, 300)
    # parent 5 wins every tournament it enters; with NaN everywhere else the
    # lower index wins, so an offspring's body comes from 5 or from a NaN pair
    k5 = tuple(par["parent"][5])
    assert sum(tuple(off["parent"][i]) == k5 for i in range(300)) > 50


def test_survivors_against_brute_force():
    rng = np.random.default_rng(4)
    for trial in range(50):
        m, l, mu = int(rng.integers(1, 30)), int(rng.integers(0, 30)), None
        fp = rng.integers(-3, 4, m).astype(np.float32)
        fo = rng.integers(-3, 4, l).astype(np.float32)
        fp[rng.random(m) < 0.2] = np.nan
        fo[rng.random(l) < 0.2] = np.nan
        mu = int(rng.integers(1, m + l + 1))
        got = E.survivors(fp, fo, mu)
        f = np.concatenate([fp, fo]).astype(np.float64)
        # brute force: every survivor beats or ties every non-survivor, ties
        # resolved towards lower positions, NaN below everything
        rank_key = [(-(x if not np.isnan(x) else -np.inf), int(np.isnan(x)), k) for k, x in enumerate(f)]
        want = sorted(k for _, _, k in sorted(rank_key)[:mu])
        assert list(got) == want


def test_tuning_moves_every_row_within_bounds_and_accepts_only_improvements():
    par = _parents(40, key=8)
    cand = E.tune_perturb(2, 11, 0, par)
    for i in range(40):
        nh = int(par["nh"][i])
        d = cand["cpg"][i, :nh] - par["cpg"][i, :nh]
        assert (np.abs(d[:, 0]) <= 0.05 + 1e-7).all()
        assert (np.abs(d[:, 1]) <= 0.25 + 1e-6).all()
        _valid(nh, cand["parent"][i], cand["face"][i], cand["axis"][i], cand["cpg"][i])
        assert (cand["cpg"][i, nh:] == 0).all()
    fb = np.linspace(0, 1, 40).astype(np.float32)
    fc = fb.copy()
    fc[::3] += 0.5
    fc[1::3] = np.nan
    out, f = E.tune_accept(par, fb, cand, fc)
    for i in range(40):
        took = i % 3 == 0
        np.testing.assert_array_equal(out["cpg"][i], cand["cpg"][i] if took else par["cpg"][i])
        assert f[i] == (fc[i] if took else fb[i])
