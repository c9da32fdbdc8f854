"""Seeded generators: determinism per (config, index), ranges and distributions."""
import numpy as np
from scipy import stats

from paper_2502_11129_amd import workloads as W


def test_determinism_per_index():
    a = W.random_trees(40)
    b = W.random_trees(10, first=30)
    s = a.subset(range(30, 40))
    for name in ("body_offset", "parent", "half_ext", "rest_quat", "axis", "cpg", "q0", "v0"):
        np.testing.assert_array_equal(getattr(s, name), getattr(b, name))
    np.testing.assert_array_equal(W.boxes(5).q0, W.boxes(5).q0)


def test_snake_layout_and_cpg_ranges():
    p = W.snake(16)
    assert p.n_variants == 16 and (p.n_bodies == 4).all()
    np.testing.assert_array_equal(p.parent[:4], [-1, 0, 1, 2])
    np.testing.assert_array_equal(p.axis[1:4], [[0, 0, 1], [0, 1, 0], [0, 0, 1]])
    cpg = p.cpg[p.parent >= 0]
    assert (cpg[:, 0] >= 0).all() and (cpg[:, 0] < 1).all()
    assert (cpg[:, 1] >= 1).all() and (cpg[:, 1] < 6).all()
    assert (cpg[:, 2] >= 0).all() and (cpg[:, 2] < 2 * np.pi).all()
    np.testing.assert_allclose(p.mass[:4], [0.15, 0.05, 0.05, 0.05])


def _depths(p, i):
    b0, b1 = p.body_offset[i], p.body_offset[i + 1]
    par = p.parent[b0:b1]
    d = np.zeros(b1 - b0, int)
    for b in range(1, b1 - b0):
        d[b] = d[par[b]] + 1
    return d


def test_random_tree_ranges_and_uniform_hinge_count():
    p = W.random_trees(2000)
    nh = p.n_hinges
    assert nh.min() >= 4 and nh.max() <= 20
    counts = np.bincount(nh, minlength=21)[4:21]
    assert stats.chisquare(counts).pvalue > 1e-3
    for i in range(0, 2000, 97):
        d = _depths(p, i)
        assert d.max() <= 4
        b0, b1 = p.body_offset[i], p.body_offset[i + 1]
        par = p.parent[b0:b1]
        assert (par[1:] < np.arange(1, b1 - b0)).all()                 # parent < child
        for b in range(1, b1 - b0):                                    # faces used once per parent
            sib = [c for c in range(1, b1 - b0) if par[c] == par[b]]
            aps = {tuple(p.anchor_parent[b0 + c]) for c in sib}
            assert len(aps) == len(sib)
        # axes: z or y in the child frame
        ax = p.axis[b0 + 1:b1]
        assert all(tuple(a) in ((0, 0, 1), (0, 1, 0)) for a in ax)


def test_quadruped_topology():
    p = W.quadrupeds(3)
    assert (p.n_hinges == 20).all()
    par = p.parent[:21]
    np.testing.assert_array_equal(par[[1, 6, 11, 16]], [0, 0, 0, 0])
    np.testing.assert_array_equal(par[2:6], [1, 2, 3, 4])
    assert (p.nv == 26).all()


def test_box_orientations_uniform_and_no_penetration():
    p = W.boxes(4000)
    q = p.q0.reshape(-1, 7)
    Q = q[:, 3:7].astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(Q, axis=1), 1.0, atol=1e-6)
    w = Q[:, 0]
    assert (w >= 0).all()
    # uniform rotations with w >= 0: E[w] = 4/(3 pi), density of w is (4/pi) sqrt(1 - w^2)
    assert abs(w.mean() - 4 / (3 * np.pi)) < 0.01
    cdf = lambda x: (2 / np.pi) * (x * np.sqrt(1 - x * x) + np.arcsin(x))
    assert stats.kstest(w, cdf).pvalue > 1e-3
    # no corner below the plane at t = 0
    half = p.half_ext.astype(np.float64)
    for i in range(0, 4000, 37):
        w_, x, y, z = Q[i]
        r2 = np.array([2 * (x * z - w_ * y), 2 * (y * z + w_ * x), 1 - 2 * (x * x + y * y)])
        assert q[i, 2] - np.abs(r2) @ half[i] >= 0.005 - 1e-6
    sides = 2 * half
    assert sides.min() >= 0.05 and sides.max() <= 0.3
    np.testing.assert_allclose(p.mass, 1000 * sides.prod(axis=1), rtol=1e-5)
    assert (p.mu >= 0.3).all() and (p.mu <= 1.2).all()


def test_genotype_robots_array_builder_equals_bodywise_builder():
    g = W.random_genotypes(700, key=31)
    a = W.population_from_genotypes(g, steps=123)
    b = W._population_from_genotypes_bodywise(g, steps=123)
    for k in ("body_offset", "parent", "half_ext", "mass", "anchor_parent", "anchor_child", "rest_quat", "axis",
              "cpg", "mu", "q0", "v0", "root_pose"):
        x, y = getattr(a, k), getattr(b, k)
        assert x.dtype == y.dtype and x.shape == y.shape and np.array_equal(x, y), k
    assert a.steps == b.steps == 123 and a.root_type == b.root_type
