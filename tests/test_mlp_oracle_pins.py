"""Pins of the surrogate oracle (CPU): BF16 rounding against known bit
patterns and torch's own conversion, GELU against torch's exact-erf GELU,
gradients against finite differences and torch autograd, Adam against its
closed-form first step and torch.optim.Adam, metrics against scipy and brute
force, features against hand-built genotypes and the robots they describe."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from paper_2502_11129_amd import workloads as WL


# ----------------------------------------------------------------------------- BF16
def test_bf16_known_values_and_ties_to_even():
    one = 1.0
    ulp = 2.0 ** -7                           # 7 stored mantissa bits
    assert M.bf16(one) == one
    assert M.bf16(one + ulp / 2) == one       # tie -> even (mantissa 0)
    assert M.bf16(one + 1.5 * ulp) == one + 2 * ulp   # tie -> even (mantissa 2)
    assert M.bf16(one + 0.51 * ulp) == one + ulp
    assert M.bf16(-3.0) == -3.0
    assert np.isnan(M.bf16(np.nan))
    assert M.bf16(np.inf) == np.inf


def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e4, 2000), rng.normal(0, 1e-6, 2000)])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


# ----------------------------------------------------------------------------- GELU
def test_gelu_against_torch_exact_erf():
    z = np.linspace(-8, 8, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(M.gelu(z), ref, rtol=1e-14, atol=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0


def test_gelu_grad_finite_difference_and_special_values():
    z = np.linspace(-6, 6, 1201)
    h = 1e-5
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, atol=1e-9)
    assert M.gelu_grad(np.array([0.0]))[0] == 0.5
    assert abs(M.gelu_grad(np.array([30.0]))[0] - 1.0) < 1e-12


# ----------------------------------------------------------------------------- MLP gradients
def _small_net(seed=3):
    W, b = M.unflatten(WL.mlp_init(seed).astype(np.float64))
    W = [w.astype(np.float64) for w in W]
    b = [x.astype(np.float64) for x in b]
    return W, b


def _loss(X, t, W, b):
    y, _ = M.forward(X, W, b, emulate_bf16=False)
    return M.mse_grad(y, t)[0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    X = rng.normal(0, 1, (6, M.N_FEAT))
    t = rng.normal(0, 1, 6)
    W, b = _small_net()
    y, cache = M.forward(X, W, b, emulate_bf16=False)
    _, dy = M.mse_grad(y, t)
    gW, gb = M.backward(cache, W, dy, emulate_bf16=False)
    h = 1e-6
    for l in range(4):
        for (i, j) in [(0, 0), (5, W[l].shape[1] - 1), (W[l].shape[0] - 1, 0), (17, W[l].shape[1] // 2)]:
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (_loss(X, t, Wp, b) - _loss(X, t, Wm, b)) / (2 * h)
            assert abs(gW[l][i, j] - fd) <= 1e-6 * max(1.0, abs(fd)), (l, i, j, gW[l][i, j], fd)
        for j in [0, b[l].shape[0] - 1]:
            bp = [x.copy() for x in b]
            bm = [x.copy() for x in b]
            bp[l][j] += h
            bm[l][j] -= h
            fd = (_loss(X, t, W, bp) - _loss(X, t, W, bm)) / (2 * h)
            assert abs(gb[l][j] - fd) <= 1e-6 * max(1.0, abs(fd))


def test_forward_backward_match_torch_autograd():
    rng = np.random.default_rng(12)
    X = rng.normal(0, 1, (32, M.N_FEAT))
    t = rng.normal(0, 1, 32)
    W, b = _small_net(4)
    y, cache = M.forward(X, W, b, emulate_bf16=False)
    loss, dy = M.mse_grad(y, t)
    gW, gb = M.backward(cache, W, dy, emulate_bf16=False)
    tW = [torch.tensor(w, requires_grad=True) for w in W]
    tb = [torch.tensor(x, requires_grad=True) for x in b]
    h = torch.tensor(X)
    for l in range(3):
        h = torch.nn.functional.gelu(h @ tW[l] + tb[l])
    ty = (h @ tW[3] + tb[3])[:, 0]
    tl = ((ty - torch.tensor(t)) ** 2).mean()
    tl.backward()
    np.testing.assert_allclose(y, ty.detach().numpy(), rtol=1e-12)
    assert abs(loss - tl.item()) < 1e-12
    for l in range(4):
        np.testing.assert_allclose(gW[l], tW[l].grad.numpy(), rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(gb[l], tb[l].grad.numpy(), rtol=1e-9, atol=1e-13)


def test_bf16_emulation_rounds_activations_and_stays_close():
    rng = np.random.default_rng(13)
    X = rng.normal(0, 1, (64, M.N_FEAT))
    W, b = M.unflatten(WL.mlp_init(1))
    y16, (hs, _) = M.forward(X, W, b, emulate_bf16=True)
    y64, _ = M.forward(X, W, b, emulate_bf16=False)
    for h in hs:
        np.testing.assert_array_equal(M.bf16(h), h)        # every stored activation is a bf16 value
    assert np.abs(y16 - y64).max() < 0.05 * max(1.0, np.abs(y64).max())


def test_mse_gradient_finite_difference():
    rng = np.random.default_rng(14)
    y, t = rng.normal(0, 1, 9), rng.normal(0, 1, 9)
    L, g = M.mse_grad(y, t)
    assert abs(L - np.mean((y - t) ** 2)) < 1e-15
    for i in range(9):
        e = np.zeros(9)
        e[i] = 1e-6
        fd = (M.mse_grad(y + e, t)[0] - M.mse_grad(y - e, t)[0]) / 2e-6
        assert abs(g[i] - fd) < 1e-8


# ----------------------------------------------------------------------------- Adam
def test_adam_first_step_closed_form():
    # bias correction makes the first step lr * g / (|g| + eps) exactly
    p = np.array([0.5, -1.0, 2.0, 0.0])
    g = np.array([0.3, -2e-3, 5.0, 0.0])
    p1, m, v = M.adam(p, g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_adam_matches_torch_optim_over_steps():
    rng = np.random.default_rng(15)
    p = rng.normal(0, 1, 50)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 8):
        g = rng.normal(0, 1, 50) * (0.1 * t)
        p, m, v = M.adam(p, g, m, v, t)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


# ----------------------------------------------------------------------------- metrics
def test_topk_tie_break_and_brute_force():
    s = np.array([1.0, 3.0, 3.0, 2.0, 3.0, 0.0])
    np.testing.assert_array_equal(M.topk_indices(s, 2), [1, 2])
    np.testing.assert_array_equal(M.topk_indices(s, 4), [1, 2, 3, 4])
    rng = np.random.default_rng(16)
    for _ in range(20):
        x = rng.integers(0, 5, 12).astype(float)
        k = int(rng.integers(1, 12))
        brute = sorted(range(12), key=lambda i: (-x[i], i))[:k]
        np.testing.assert_array_equal(M.topk_indices(x, k), sorted(brute))


def test_recall_extremes():
    x = np.arange(1000.0)
    assert M.recall_at(x, x) == 1.0
    assert M.recall_at(-x, x) == 0.0
    assert M.recall_at(x + 0.5 * (x % 2), x) == 1.0          # order-preserving inside the top 5 %


def test_spearman_against_scipy_and_ties():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(17)
    a = rng.normal(0, 1, 300)
    b = a + rng.normal(0, 1, 300)
    assert abs(M.spearman(a, b) - spearmanr(a, b).statistic) < 1e-12
    a = rng.integers(0, 5, 200).astype(float)
    b = rng.integers(0, 7, 200).astype(float)
    assert abs(M.spearman(a, b) - spearmanr(a, b).statistic) < 1e-12
    assert abs(M.spearman(a, 3 * a + 1) - 1.0) < 1e-12


# ----------------------------------------------------------------------------- features
def _one(nh, parent, face, axis, cpg):
    g = WL._empty_genotypes(1)
    g.nh[0] = nh
    g.parent[0, :nh] = parent
    g.face[0, :nh] = face
    g.axis[0, :nh] = axis
    g.cpg[0, :nh] = cpg
    return g


def test_features_hand_case():
    # core -> brick1 (+x, z axis) -> brick2 (+y, y axis); core -> brick3 (-y, z axis)
    cpg = [[0.5, 3.0, math.pi], [0.25, 6.0, 0.0], [1.0, 1.5, math.pi / 2]]
    g = _one(3, [0, 1, 0], [0, 2, 3], [0, 1, 0], cpg)
    F = M.features(g)[0]
    exp = np.zeros(128)
    exp[0:3] = [0.5, 0.25, 1.0]
    exp[20:23] = [0.5, 1.0, 0.25]
    exp[40:43] = [0.5, 0.0, 0.25]
    exp[60:63] = [1, -1, 1]
    exp[80:83] = [0.25, 0.5, 0.25]
    exp[100:104] = [3 / 20, 2 / 20, 1 / 20, 0.5]
    exp[104:109] = [2 / 20, 1 / 20, 0, 0, 0]
    exp[109:114] = [0.25, 0.25, 0, 0, 0]               # limbs of sizes 1 and 2
    exp[114:118] = [1, 0, 0, 1]
    np.testing.assert_allclose(F, exp, rtol=0, atol=1e-7)


def test_features_agree_with_the_robots_they_describe():
    """Depth counts and limb sizes recomputed from the robots' own parent
    arrays (the simulator input), not from the genotype."""
    g = WL.random_genotypes(300, key=7)
    F = M.features(g)
    pop = WL.population_from_genotypes(g)
    for i in range(300):
        b0, b1 = pop.body_offset[i], pop.body_offset[i + 1]
        par = pop.parent[b0:b1]
        depth = np.zeros(b1 - b0, int)
        for b in range(1, b1 - b0):
            depth[b] = depth[par[b]] + 1
        counts = np.bincount(depth[1:], minlength=6)[1:6] / 20.0
        np.testing.assert_allclose(F[i, 104:109], counts)
        assert F[i, 103] == depth.max() / 4.0
        assert F[i, 100] == (b1 - b0 - 1) / 20.0
        # limb = set of bodies whose path to the core passes through a core child
        sizes = []
        for c in np.where(par == 0)[0]:
            n = 0
            for b in range(1, b1 - b0):
                a = b
                while par[a] != 0:
                    a = par[a]
                n += a == c
            sizes.append(n)
        hist = np.zeros(5)
        for s in sizes:
            hist[[1, 2, 4, 8, 10**9].index(next(x for x in [1, 2, 4, 8, 10**9] if s <= x))] += 0.25
        np.testing.assert_allclose(F[i, 109:114], hist)
        assert F[i, 118:].sum() == 0
        assert depth.max() <= 4


def test_genotypes_reproduce_the_tree_population():
    g = WL.tree_genotypes(range(10))
    p = WL.population_from_genotypes(g)
    q = WL.random_trees(10)
    for a in ("body_offset", "parent", "anchor_parent", "anchor_child", "rest_quat", "axis", "cpg", "q0", "v0"):
        np.testing.assert_array_equal(getattr(p, a), getattr(q, a))


def test_flat_layout_round_trip_and_init_ranges():
    p = WL.mlp_init(0)
    assert p.shape == (164865,) and p.dtype == np.float32
    Wl, bl = M.unflatten(p)
    assert [w.shape for w in Wl] == [(128, 256), (256, 256), (256, 256), (256, 1)]
    np.testing.assert_array_equal(M.flatten(Wl, bl), p)
    assert np.abs(Wl[0]).max() <= 1 / np.sqrt(128) and np.abs(Wl[1]).max() <= 1 / 16
    assert np.abs(Wl[0]).max() > 0.9 / np.sqrt(128)


def test_standardize_moments():
    rng = np.random.default_rng(18)
    y = rng.gamma(2.0, 0.1, 5000)
    z, mu, sd = M.standardize(y)
    assert abs(z.mean()) < 1e-12 and abs(z.std() - 1.0) < 1e-12
    assert abs(mu - np.mean(y)) < 1e-12 and abs(sd - np.std(y)) < 1e-12
    z, mu, sd = M.standardize(np.full(10, 3.0))
    assert (z == 0).all() and sd == 0
