"""FP64 reference of the learned surrogate -- TEST INFRASTRUCTURE ONLY.

Imported by tests/ (and nothing on the product path).  Plain numpy:

* genotype features (128 values per candidate, layout below);
* an MLP 128 -> 256 -> 256 -> 256 -> 1 with GELU (x Phi(x), exact erf;
  Hendrycks & Gimpel 2016), optionally emulating BF16 storage with
  round-to-nearest-even at the same points as the GPU kernels: inputs,
  weight copies, every hidden activation and every hidden-layer gradient that
  feeds a matrix product;
* target standardisation, its backward pass, the mean-squared-error loss, Adam (Kingma & Ba 2015,
  beta = (0.9, 0.999), eps = 1e-8) with FP32 master weights;
* screening metrics: top-5% recall (ties broken by lower index) and
  Spearman's rho (Pearson correlation of average ranks).

Feature layout (float, 128 per candidate; hinge j drives body j + 1):
  [0,20) A_j   [20,40) omega_j / 6   [40,60) phi_j / 2 pi   (zero padded)
  [60,80) axis: +1 hinge about child z, -1 about child y, 0 padding
  [80,100) depth of body j+1 / 4
  100 nh/20, 101 n_z/20, 102 n_y/20, 103 max depth/4
  [104,109) number of bodies at depth 1..5, / 20
  [109,114) sizes of the subtrees hanging off the core (limbs), histogram
            over {1, 2, 3-4, 5-8, >= 9}, / 4
  [114,118) core faces +x, -x, +y, -y occupied (0/1)
  [118,128) zero
"""
from __future__ import annotations

import math

import numpy as np

MAX_H = 20
N_FEAT = 128
HIDDEN = 256


# ----------------------------------------------------------------------------- BF16
def bf16(x):
    """Round to bfloat16 (round-to-nearest-even on the float32 value), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------- features
def features(g) -> np.ndarray:
    """Features of genotypes (object with nh [N], parent [N,20], face [N,20],
    axis [N,20], cpg [N,20,3]), one candidate at a time."""
    n = len(g.nh)
    F = np.zeros((n, N_FEAT), dtype=np.float64)
    for i in range(n):
        nh = int(g.nh[i])
        depth = [0]
        for j in range(nh):
            depth.append(depth[int(g.parent[i, j])] + 1)
        for j in range(nh):
            A, om, ph = (float(x) for x in g.cpg[i, j])
            F[i, j] = A
            F[i, 20 + j] = om / 6.0
            F[i, 40 + j] = ph / (2 * math.pi)
            F[i, 60 + j] = 1.0 if int(g.axis[i, j]) == 0 else -1.0
            F[i, 80 + j] = depth[j + 1] / 4.0
        nz = sum(1 for j in range(nh) if int(g.axis[i, j]) == 0)
        F[i, 100] = nh / 20.0
        F[i, 101] = nz / 20.0
        F[i, 102] = (nh - nz) / 20.0
        F[i, 103] = max(depth) / 4.0
        for dd in range(1, 6):
            F[i, 103 + dd] = sum(1 for x in depth[1:] if x == dd) / 20.0
        # limb sizes: subtree sizes of the core's children
        size = [1] * (nh + 1)
        for b in range(nh, 0, -1):
            p = int(g.parent[i, b - 1])
            if p > 0:
                size[p] += size[b]
        for b in range(1, nh + 1):
            if int(g.parent[i, b - 1]) == 0:
                s = size[b]
                k = 0 if s == 1 else 1 if s == 2 else 2 if s <= 4 else 3 if s <= 8 else 4
                F[i, 109 + k] += 0.25
                F[i, 114 + int(g.face[i, b - 1])] = 1.0
    return F


# ----------------------------------------------------------------------------- MLP
def gelu(z):
    from scipy.special import erf
    return z * 0.5 * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unflatten(p):
    """Flat parameter vector (W1, b1, W2, b2, W3, b3, W4, b4; W_l[in][out]
    row-major) -> lists W, b (views, dtype kept)."""
    dims = [N_FEAT, HIDDEN, HIDDEN, HIDDEN, 1]
    W, b, o = [], [], 0
    for l in range(4):
        n = dims[l] * dims[l + 1]
        W.append(p[o:o + n].reshape(dims[l], dims[l + 1]))
        o += n
        b.append(p[o:o + dims[l + 1]])
        o += dims[l + 1]
    assert o == len(p)
    return W, b


def flatten(W, b):
    return np.concatenate([x for l in range(4) for x in (np.ravel(W[l]), np.ravel(b[l]))])


def forward(X, W, b, emulate_bf16=True):
    """Returns (prediction [B], cache).  Hidden layers: z = h W + b, h' = GELU(z)."""
    r = bf16 if emulate_bf16 else (lambda x: np.asarray(x, np.float64))
    h = r(X)
    hs, zs = [h], []
    for l in range(3):
        z = h @ r(W[l]).astype(np.float64) + b[l].astype(np.float64)
        zs.append(z)
        h = r(gelu(z))
        hs.append(h)
    y = h @ r(W[3]).astype(np.float64)[:, 0] + float(b[3][0])
    return y, (hs, zs)


def backward(cache, W, dy, emulate_bf16=True, return_dz=False):
    """Gradients of sum(dy * y) w.r.t. W and b (float64).  With return_dz,
    also the output gradient of each layer (dz, after its rounding; the
    head's is dy), whose products with the layer inputs make up the sums."""
    r = bf16 if emulate_bf16 else (lambda x: np.asarray(x, np.float64))
    hs, zs = cache
    gW, gb, dzs = [None] * 4, [None] * 4, [None] * 4
    gW[3] = (hs[3].T @ dy)[:, None]
    gb[3] = np.array([dy.sum()])
    dzs[3] = np.asarray(dy, np.float64)[:, None]
    dh = np.outer(dy, r(W[3]).astype(np.float64)[:, 0])
    for l in (2, 1, 0):
        dz = r(dh * gelu_grad(zs[l]))
        dzs[l] = dz
        gW[l] = hs[l].T @ dz
        gb[l] = dz.sum(axis=0)
        if l > 0:
            dh = dz @ r(W[l]).astype(np.float64).T
    if return_dz:
        return gW, gb, dzs
    return gW, gb


def standardize(y):
    """(y - mean) / std with the population std (1 when zero); returns (z, mean, std)."""
    y = np.asarray(y, np.float64)
    mean = y.mean()
    sd = np.sqrt(np.mean((y - mean) ** 2))
    return (y - mean) / (sd if sd > 0 else 1.0), mean, sd


def mse_grad(y, t):
    """Loss mean((y - t)^2) and its gradient w.r.t. y."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / len(d)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on float64 copies; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------- metrics
def topk_indices(scores, k):
    """Indices of the k largest scores; ties broken by lower index."""
    order = np.lexsort((np.arange(len(scores)), -np.asarray(scores)))
    return np.sort(order[:k])


def recall_at(pred, true, frac=0.05):
    k = max(1, int(round(frac * len(true))))
    a = set(topk_indices(pred, k).tolist())
    b = set(topk_indices(true, k).tolist())
    return len(a & b) / k


def spearman(x, y):
    from scipy.stats import rankdata
    rx, ry = rankdata(x), rankdata(y)
    rx -= rx.mean()
    ry -= ry.mean()
    return float((rx * ry).sum() / np.sqrt((rx * rx).sum() * (ry * ry).sum()))
