"""GPU parity of the evolutionary-loop kernels (through the C ABI) against
the reference operators of oracle/ea_oracle.py on the same seeded inputs:
variation, Lamarckian perturbation and acceptance, gathering and survivor
selection are integer or explicitly rounded float32 work, so the bar is
bit-exact equality.  A small end-to-end run checks the loop's invariants."""
import sys

import numpy as np
import pytest

from oracle import ea_oracle as E
from paper_2502_11129_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _np(g):
    return dict(nh=g.nh.astype(np.int32), parent=g.parent.astype(np.int32), face=g.face.astype(np.int32),
                axis=g.axis.astype(np.int32), cpg=g.cpg.astype(np.float32))


def _dev(d):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v, np.int8 if k in ("parent", "face", "axis") else
                                                     (np.int32 if k == "nh" else np.float32))).cuda()
            for k, v in d.items()}


def _host(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _same(got, want):
    for k in ("nh", "parent", "face", "axis"):
        np.testing.assert_array_equal(got[k].astype(np.int64), want[k].astype(np.int64), err_msg=k)
    np.testing.assert_array_equal(got["cpg"].view(np.uint32), want["cpg"].astype(np.float32).view(np.uint32))


def _fitness(n, rng):
    f = np.round(rng.normal(0.1, 0.1, n), 2).astype(np.float32)   # many ties
    f[rng.random(n) < 0.05] = np.nan
    return f


@pytest.mark.parametrize("mu, n_off, seed, gen", [(512, 3001, 0x123456789ABCDEF0, 0), (97, 1000, 7, 5),
                                                  (1, 130, 42, 3)])
def test_vary_bit_exact(mu, n_off, seed, gen):
    import torch
    from paper_2502_11129_amd import ea as EA
    _say(f"[ea_vary] mu {mu}, offspring {n_off}, seed {seed:#x}, generation {gen}")
    par = _np(W.random_genotypes(mu, key=21))
    fit = _fitness(mu, np.random.default_rng(mu))
    got = _host(EA.vary(_dev(par), torch.from_numpy(fit).cuda(), n_off, seed, gen))
    want = E.vary(gen, seed, par, fit, n_off)
    _same(got, want)
    assert ((got["nh"] >= 4) & (got["nh"] <= 20)).all()
    if mu > 1:
        assert len(set(got["nh"].tolist())) > 5


def test_tune_perturb_and_accept_bit_exact():
    import torch
    from paper_2502_11129_amd import ea as EA
    base = _np(W.random_genotypes(777, key=22))
    d = _dev(base)
    cand = EA.tune_perturb(d, 99, 4, 1).cpu().numpy()
    want = E.tune_perturb(4, 99, 1, base)
    np.testing.assert_array_equal(cand.view(np.uint32), want["cpg"].view(np.uint32))
    rng = np.random.default_rng(3)
    fb = _fitness(777, rng)
    fc = _fitness(777, rng)
    fb_d, fc_d = torch.from_numpy(fb.copy()).cuda(), torch.from_numpy(fc).cuda()
    cb = d["cpg"].clone()
    EA.tune_accept(cb, fb_d, torch.from_numpy(cand).cuda(), fc_d)
    out, f = E.tune_accept(base, fb, want, fc)
    np.testing.assert_array_equal(cb.cpu().numpy().view(np.uint32), out["cpg"].view(np.uint32))
    np.testing.assert_array_equal(fb_d.cpu().numpy().view(np.uint32), f.view(np.uint32))


def test_survivors_and_gather_exact():
    import torch
    from paper_2502_11129_amd import ea as EA
    from paper_2502_11129_amd.surrogate import Surrogate
    sur = Surrogate(max_batch=64)
    rng = np.random.default_rng(8)
    a = _np(W.random_genotypes(300, key=23))
    b = _np(W.random_genotypes(257, key=24))
    fa, fb = _fitness(300, rng), _fitness(257, rng)
    idx = sur.topk(torch.from_numpy(np.concatenate([fa, fb])).cuda(), 300)
    want_idx = E.survivors(fa, fb, 300)
    np.testing.assert_array_equal(idx.cpu().numpy(), want_idx)
    # gather, with out-of-range positions written as padding with NaN fitness
    pos = np.concatenate([want_idx, [-1, 557, 10 ** 6]]).astype(np.int32)
    g, f = EA.gather(torch.from_numpy(pos).cuda(), _dev(a), torch.from_numpy(fa).cuda(), _dev(b),
                     torch.from_numpy(fb).cuda())
    g, f = _host(g), f.cpu().numpy()
    cat = {k: np.concatenate([a[k], b[k]]) for k in a}
    fcat = np.concatenate([fa, fb])
    want = {k: v[want_idx] for k, v in cat.items()}
    _same({k: v[:300] for k, v in g.items()}, want)
    np.testing.assert_array_equal(f[:300].view(np.uint32), fcat[want_idx].view(np.uint32))
    assert (g["nh"][300:] == 0).all() and (g["parent"][300:] == -1).all() and np.isnan(f[300:]).all()
    sur.close()


def test_small_evolution_run_invariants():
    """Two generations of the whole loop (16 parents, 16 offspring screened
    from 64, one tuning round, 300 steps): parents stay valid trees, the best
    fitness never drops (elitist survivors) and offspring enter the parents."""
    from paper_2502_11129_amd import evolution as EV
    out = EV.run(generations=2, mu=16, lam=16, screen=4, T=300, tune_rounds=1, pretrain=256, epochs=2, seed=5,
                 log=_say)
    h = out["history"]
    assert len(h) == 2 and h[1]["best"] >= h[0]["best"]
    assert all(np.isfinite(r["best"]) for r in h)
    assert out["generations_per_s"] > 0
