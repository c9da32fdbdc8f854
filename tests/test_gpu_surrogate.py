"""GPU parity of the surrogate kernels against the FP64 surrogate oracle
(BF16-emulating at the same rounding points), through the C ABI.

Bars: features bit-exact; top-k indices exact; forward predictions within
1e-3 relative norm-wise and, element by element, |got - ref| <= 1e-2 |ref| +
1e-3 rms(ref); parameter gradients within 1e-3 relative norm-wise per tensor
and, element by element, within the bound of the BF16 arithmetic (see
_grad_bar: FP32 accumulation order and occasional one-ulp BF16 rounding
differences of the operands are the only expected deviations, and a flipped
BF16 operand moves a gradient entry by at most one BF16 ulp of one term of its
sum); Adam within 1e-6 relative of the FP64 formula."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_2502_11129_amd import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _sur(**kw):
    from paper_2502_11129_amd.surrogate import Surrogate
    return Surrogate(**kw)


def _bits(X):
    """BF16 device tensor -> uint16 host bit patterns."""
    import torch
    return X.cpu().view(torch.int16).numpy().view(np.uint16)


def _oracle_bits(F):
    return (M.bf16(F).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30)


ELEM_REL, ELEM_RMS = 1e-2, 1e-3


# A gradient entry g_ij = sum_b h_bi dz_bj (h the layer input, dz its output
# gradient, both BF16 in the kernels and in the emulating oracle).  The two
# sides round the same FP64/FP32 quantities to BF16, so an operand can land on
# the neighbouring BF16 value when the unrounded values differ near a rounding
# boundary; each such flip moves the products it enters by one BF16 ulp
# (<= 2^-7 of the operand).  FLIPS flips of the largest term of an entry's sum
# are allowed, plus the FP32 accumulation-order term sqrt(B) 2^-24 sum_b |h dz|
# (probabilistic rounding-error bound of a B-term sum) and the 1e-2 relative
# part of the element bar.
FLIPS = 4


def _grad_bar(h, dz, ref):
    """Per-element bound for the gradient h^T dz (ref: the oracle's value)."""
    h = np.abs(np.asarray(h, np.float64))
    dz = np.abs(np.asarray(dz, np.float64))
    B = h.shape[0]
    big = np.zeros((h.shape[1], dz.shape[1]))
    for s in range(0, B, 64):
        big = np.maximum(big, np.max(h[s:s + 64, :, None] * dz[s:s + 64, None, :], axis=0))
    return ELEM_REL * np.abs(ref) + FLIPS * 2.0 ** -7 * big + np.sqrt(B) * 2.0 ** -24 * (h.T @ dz)


def _ratio(got, ref, bar):
    """Largest |got - ref| / bar; an entry with a zero bound (every term of
    its sum zero, e.g. a feature that is zero in every row) must be exact."""
    d = np.abs(np.asarray(got, np.float64) - ref)
    return float(np.max(np.where(bar > 0, d / np.where(bar > 0, bar, 1.0), np.where(d > 0, np.inf, 0.0))))


def _elem(a, b):
    """Largest |a - b| / (ELEM_REL |b| + ELEM_RMS rms(b)) over the elements."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b))
    return float(np.max(np.abs(a - b) / (ELEM_REL * np.abs(b) + ELEM_RMS * rms + 1e-30)))


def test_features_bit_exact(torch):
    g = W.random_genotypes(3001, key=11)            # ragged: not a multiple of the 64-thread block
    gt = W.tree_genotypes(range(200))
    _say("[features] 3001 random + 200 tree genotypes")
    s = _sur()
    for gg in (g, gt):
        X = s.features(s.upload_genotypes(gg))
        ref = _oracle_bits(M.features(gg))
        got = _bits(X)
        assert got.shape == ref.shape
        np.testing.assert_array_equal(got, ref)


def test_features_invalid_rows_are_nan(torch):
    g = W.random_genotypes(6, key=12)
    g.nh[1] = 0                   # nh out of range
    g.parent[2, 3] = 9            # parent not earlier than the child
    g.face[3, 0] = 4              # face out of range
    g.axis[4, 1] = 2              # axis flag out of range
    s = _sur()
    X = s.features(s.upload_genotypes(g)).float().cpu().numpy()
    for i in (1, 2, 3, 4):
        assert np.isnan(X[i]).all(), i
    assert np.isfinite(X[[0, 5]]).all()


def test_forward_matches_oracle_and_gathers(torch):
    g = W.random_genotypes(1000, key=13)
    p = W.mlp_init(3)
    Wl, bl = M.unflatten(p)
    Xref = M.bf16(M.features(g))
    yref, _ = M.forward(Xref, Wl, bl, emulate_bf16=True)
    _say("[forward] 1000 rows, 3 hidden layers")
    s = _sur(params=p)
    X = s.features(s.upload_genotypes(g))
    y = s.predict(X).cpu().numpy()
    e, r = _rel(y, yref), _elem(y, yref)
    _say(f"  relative error {e:.2e}, max abs {np.abs(y - yref).max():.2e}, element ratio {r:.3f}")
    assert e <= REL and r <= 1.0
    # gathered rows give the same values bit for bit (rows are independent)
    idx = np.random.default_rng(0).permutation(1000)[:333].astype(np.int32)
    yg = s.predict(X, torch.from_numpy(idx).cuda()).cpu().numpy()
    np.testing.assert_array_equal(yg, y[idx])


def test_forward_beyond_one_chunk(torch):
    """More rows than one forward chunk (65536): sampled rows against the oracle."""
    n = 70001
    rng = np.random.default_rng(14)
    Xh = rng.normal(0, 1, (n, 128)).astype(np.float32)
    p = W.mlp_init(4)
    s = _sur(params=p)
    X = torch.from_numpy(Xh).to(torch.bfloat16).cuda()
    y = s.predict(X).cpu().numpy()
    rows = np.concatenate([rng.choice(n, 400, replace=False), [0, 65535, 65536, n - 1]])
    Wl, bl = M.unflatten(p)
    yref, _ = M.forward(Xh[rows], Wl, bl, emulate_bf16=True)
    e, r = _rel(y[rows], yref), _elem(y[rows], yref)
    _say(f"[forward] n={n}: sampled relative error {e:.2e}, element ratio {r:.3f}")
    assert e <= REL and r <= 1.0


def _grads_case(torch, B, seed):
    n = B + 37
    g = W.random_genotypes(n, key=seed)
    p = W.mlp_init(seed)
    rng = np.random.default_rng(seed)
    target = rng.normal(0, 1, n).astype(np.float32)
    idx = rng.permutation(n)[:B].astype(np.int32)
    Wl, bl = M.unflatten(p)
    Xref = M.bf16(M.features(g))
    y, cache = M.forward(Xref[idx], Wl, bl, emulate_bf16=True)
    loss, dy = M.mse_grad(y, target[idx].astype(np.float64))
    gW, gb, dzs = M.backward(cache, Wl, dy, emulate_bf16=True, return_dz=True)
    s = _sur(params=p, max_batch=max(B, 64))
    X = s.features(s.upload_genotypes(g))
    lt = s.train_step(X, torch.from_numpy(target).cuda(), torch.from_numpy(idx).cuda())
    return s, p, loss, float(lt.item()), gW, gb, s.grad(), cache[0], dzs


@pytest.mark.parametrize("B", [4096, 1000])
def test_train_step_gradients_match_oracle(torch, B):
    _say(f"[backward] batch {B}")
    s, p, loss, loss_gpu, gW, gb, gg, hs, dzs = _grads_case(torch, B, 20 + B % 7)
    assert abs(loss_gpu - loss) <= REL * loss
    Wg, bg = M.unflatten(gg)
    for l in range(4):
        ew, eb = _rel(Wg[l], gW[l]), _rel(bg[l], gb[l])
        barW = _grad_bar(hs[l], dzs[l], gW[l])
        barb = _grad_bar(np.ones((hs[l].shape[0], 1)), dzs[l], gb[l][None, :])[0]
        rw, rb = _ratio(Wg[l], gW[l], barW), _ratio(bg[l], gb[l], barb)
        _say(f"  layer {l + 1}: grad W rel {ew:.2e} (element ratio {rw:.3f}), grad b rel {eb:.2e} ({rb:.3f})")
        assert ew <= REL and eb <= REL
        assert rw <= 1.0 and rb <= 1.0
    # the step that followed used Adam's first update, lr * g / (|g| + eps)
    p1, m1, v1, t = s.get_state()
    assert t == 1
    g_ref = M.flatten(gW, gb)
    m_ref = 0.1 * g_ref
    np.testing.assert_allclose(m1, m_ref, rtol=0, atol=REL * np.abs(g_ref).max())
    step = p1.astype(np.float64) - p
    big = np.abs(g_ref) > 1e-3 * np.abs(g_ref).max()
    np.testing.assert_allclose(step[big], -1e-3 * np.sign(g_ref[big]), rtol=1e-3)


def test_adam_step_matches_formula(torch):
    rng = np.random.default_rng(30)
    p0 = W.mlp_init(5)
    m0 = rng.normal(0, 0.01, p0.shape).astype(np.float32)
    v0 = rng.uniform(0, 1e-3, p0.shape).astype(np.float32)
    g = rng.normal(0, 0.05, p0.shape).astype(np.float32)
    s = _sur(params=p0)
    s.set_state(p0, m0, v0, t=6)
    s.adam_step(torch.from_numpy(g).cuda())
    p1, m1, v1, t = s.get_state()
    pr, mr, vr = M.adam(p0.astype(np.float64), g.astype(np.float64), m0.astype(np.float64), v0.astype(np.float64), 7)
    assert t == 7
    # FP32 rounding of each term of the moment updates
    assert (np.abs(m1 - mr) <= 4e-7 * (0.9 * np.abs(m0) + 0.1 * np.abs(g)) + 1e-30).all()
    assert (np.abs(v1 - vr) <= 4e-7 * (0.999 * v0 + 0.001 * g.astype(np.float64) ** 2) + 1e-30).all()
    # the update to 1e-6 of itself, plus the final rounding of p to float
    upd = pr - p0
    assert (np.abs(p1 - pr) <= 1e-6 * np.abs(upd) + 1.2e-7 * np.abs(pr) + 1e-12).all()
    # the BF16 weight copies follow the new masters
    Xh = rng.normal(0, 1, (300, 128)).astype(np.float32)
    y = s.predict(torch.from_numpy(Xh).to(torch.bfloat16).cuda()).cpu().numpy()
    Wl, bl = M.unflatten(p1)
    yref, _ = M.forward(Xh, Wl, bl, emulate_bf16=True)
    assert _rel(y, yref) <= REL


def test_topk_exact_with_ties_nan_and_signed_zero(torch):
    rng = np.random.default_rng(40)
    n = 1_000_003
    sc = np.round(rng.normal(0, 1, n), 2).astype(np.float32)      # many ties
    sc[rng.choice(n, 1000, replace=False)] = np.nan
    sc[rng.choice(n, 500, replace=False)] = -0.0
    sc[rng.choice(n, 500, replace=False)] = 0.0
    sc[rng.choice(n, 10, replace=False)] = np.inf
    sc[rng.choice(n, 10, replace=False)] = -np.inf
    s = _sur()
    d = torch.from_numpy(sc).cuda()
    # reference order: score descending (-0 == +0), NaN below -inf, then index
    val = np.where(np.isnan(sc), -np.inf, sc).astype(np.float64)
    order = np.lexsort((np.arange(n), np.isnan(sc), -val))
    for k in (50000, 1, 12345, n):
        _say(f"[topk] n={n} k={k}")
        got = s.topk(d, k).cpu().numpy()
        np.testing.assert_array_equal(got, np.sort(order[:k]).astype(np.int32))
    # the oracle's own rule on a NaN-free copy
    clean = np.where(np.isnan(sc), -3e38, sc).astype(np.float32)
    got = s.topk(torch.from_numpy(clean).cuda(), 50000).cpu().numpy()
    np.testing.assert_array_equal(got, M.topk_indices(clean, 50000))
    # small and degenerate sizes
    for m, k in ((1, 1), (5, 3), (1025, 1024), (4096, 7)):
        x = np.zeros(m, np.float32)
        got = s.topk(torch.from_numpy(x).cuda(), k).cpu().numpy()
        np.testing.assert_array_equal(got, np.arange(k))


def test_standardize_matches_oracle(torch):
    rng = np.random.default_rng(50)
    y = rng.gamma(2.0, 0.05, 200000).astype(np.float32)
    s = _sur()
    z, mu, sd = s.standardize(torch.from_numpy(y).cuda())
    zr, mur, sdr = M.standardize(y)
    assert abs(mu - mur) <= 1e-9 * abs(mur) and abs(sd - sdr) <= 1e-9 * sdr
    np.testing.assert_allclose(z.cpu().numpy(), zr, rtol=1e-6, atol=1e-6)


def test_training_reduces_loss(torch):
    """A learnable synthetic target (a fixed smooth function of the features)."""
    from paper_2502_11129_amd.surrogate import train
    g = W.random_genotypes(8192, key=60)
    F = M.features(g)
    t = (np.sin(3 * F[:, 0]) + F[:, 100] * 2 - F[:, 109] + 0.5 * F[:, 20] * F[:, 40]).astype(np.float32)
    s = _sur(params=W.mlp_init(6))
    X = s.features(s.upload_genotypes(g))
    z, _, _ = s.standardize(torch.from_numpy(t).cuda())
    losses = train(s, X, z, epochs=40, batch=1024, seed=1)
    first, last = losses[0].mean(), losses[-1].mean()
    _say(f"[train] loss {first:.4f} -> {last:.4f}")
    assert np.isfinite(losses).all()
    assert last < 0.25 * first


def test_out_of_range_index_gives_nan_not_a_fault(torch):
    rng = np.random.default_rng(70)
    Xh = rng.normal(0, 1, (100, 128)).astype(np.float32)
    s = _sur()
    X = torch.from_numpy(Xh).to(torch.bfloat16).cuda()
    idx = torch.tensor([0, -1, 5, 100, 99], dtype=torch.int32).cuda()
    y = s.predict(X, idx).cpu().numpy()
    assert np.isnan(y[[1, 3]]).all() and np.isfinite(y[[0, 2, 4]]).all()
