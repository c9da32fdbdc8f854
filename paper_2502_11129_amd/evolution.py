"""Evolutionary outer loop on one MI355X: a (mu + lambda) evolution of robot
bodies and CPG controllers with a learned pre-screen and Lamarckian
controller tuning, every operator in the HIP library (include/ea.h,
include/sur.h, include/sim.h).

The paper's motivation (Sec. 1): in evolutionary robotics with Revolve2 the
physics simulation is most of the run time, and memetic (Lamarckian)
variants multiply it.  One generation here:

  1. variation      screen x lambda offspring of the mu parents (binary
                    tournaments, controller crossover, body and controller
                    mutation)                                        ea_vary
  2. pre-screen     features and surrogate predictions of every offspring,
                    the lambda best predictions kept    sur_features/predict/topk, ea_gather
  3. evaluation     exact rollouts of the kept offspring (T steps); the
                    simulator is the judge                            sim_rollout
  4. Lamarckian     per round: every kept controller perturbed, rolled out
     tuning         again, the better controller (and its fitness) kept and
                    written back into the genotype        ea_tune_perturb/accept
  5. survivors      the mu best of parents and offspring     sur_topk, ea_gather
  6. surrogate      one epoch on the new (features, fitness) pairs  sur_train_epoch

Only the conversion of genotypes into simulator models (array assembly and
sim_create's packing) runs on the host.

Usage: python -m paper_2502_11129_amd.evolution [--generations 8] [--mu 4096] [--lam 4096] ...
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ea as EA
from . import surrogate as SU
from . import workloads as W
from .sim import Simulator


def to_host(geno) -> W.Genotypes:
    h = {k: v.cpu().numpy() for k, v in geno.items()}
    return W.Genotypes(h["nh"].astype(np.int32), h["parent"].astype(np.int32), h["face"].astype(np.int32),
                       h["axis"].astype(np.int32), h["cpg"].astype(np.float32))


def to_device(g: W.Genotypes, device):
    import torch
    return {k: torch.from_numpy(v).to(device) for k, v in W.genotype_arrays(g).items()}


class Evaluator:
    """Exact fitness of device genotypes: models assembled on the host, one
    rollout of T steps on the GPU; reports GPU (events) and host seconds."""

    def __init__(self, T, device):
        self.T, self.device = T, device
        self.gpu_s = self.host_s = 0.0

    def __call__(self, geno, cpg=None):
        import torch
        t0 = time.perf_counter()
        g = to_host(geno)
        if cpg is not None:
            g.cpg = cpg.cpu().numpy().astype(np.float32)
        sim = Simulator(W.population_from_genotypes(g, steps=self.T), device=self.device)
        self.host_s += time.perf_counter() - t0
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        sim.rollout(self.T)
        f = sim.fitness_device()
        e1.record(st)
        e1.synchronize()
        self.gpu_s += e0.elapsed_time(e1) / 1e3
        sim.close()
        return f


def run(generations=8, mu=4096, lam=4096, screen=8, T=5000, tune_rounds=1, pretrain=20000, epochs=30, seed=2025,
        log=print):
    import torch
    dev = torch.device("cuda")
    t_start = time.perf_counter()
    ev = Evaluator(T, dev)
    # initial parents and their exact fitness
    parents = to_device(W.random_genotypes(mu, key=500), dev)
    fit = ev(parents)
    # surrogate pre-trained on labelled random robots (targets standardised once)
    sur = SU.Surrogate(seed=seed, max_batch=4096)
    if pretrain:
        pre = W.random_genotypes(pretrain, key=501)
        y, _, _ = SU.simulate_fitness(pre, T=T)
        X = sur.features(to_device(pre, dev))
        yd = torch.from_numpy(y).to(dev)
        ys, mean, std = sur.standardize(yd)
        SU.train(sur, X, ys, epochs, seed=seed)
    else:
        mean, std = 0.0, 1.0
    std = std or 1.0
    setup_s = time.perf_counter() - t_start
    log(json.dumps({"setup_s": setup_s, "mu": mu, "lam": lam, "screen": screen, "T": T, "tune_rounds": tune_rounds,
                    "best": float(torch.nan_to_num(fit, nan=-1.0).max()), "mean": float(fit.nanmean())}))
    history = []
    t_loop = time.perf_counter()
    for gen in range(generations):
        ev.gpu_s = ev.host_s = 0.0
        ph = {}
        t0 = time.perf_counter()
        pool = EA.vary(parents, fit, screen * lam, seed, gen)                       # 1
        X = sur.features(pool)                                                     # 2
        pred = sur.predict(X)
        keep = sur.topk(pred, lam)
        kept, _ = EA.gather(keep, pool, with_fitness=False)
        torch.cuda.synchronize()
        ph["vary_screen_s"] = time.perf_counter() - t0
        f_off = ev(kept)                                                           # 3
        for r in range(tune_rounds):                                               # 4
            cand = EA.tune_perturb(kept, seed, gen, r)
            f_cand = ev(kept, cand)
            EA.tune_accept(kept["cpg"], f_off, cand, f_cand)
        ph["eval_gpu_s"], ph["eval_host_s"] = ev.gpu_s, ev.host_s
        t1 = time.perf_counter()
        f_all = torch.cat([fit, f_off])                                            # 5
        surv = sur.topk(f_all, mu)
        parents, fit = EA.gather(surv, parents, fit, kept, f_off)
        Xk = sur.features(kept)                                                    # 6
        yk = torch.nan_to_num((f_off - mean) / std, nan=0.0)
        perm = torch.from_numpy(np.random.default_rng([9, seed, gen]).permutation(lam).astype(np.int32)).to(dev)
        sur.train_epoch(Xk, yk, perm, min(4096, lam))
        torch.cuda.synchronize()
        ph["select_train_s"] = time.perf_counter() - t1
        ph["generation_s"] = time.perf_counter() - t0
        rec = dict(generation=gen, best=float(torch.nan_to_num(fit, nan=-1.0).max()), mean=float(fit.nanmean()),
                   offspring_mean=float(f_off.nanmean()), survivors_from_offspring=int((surv >= mu).sum()), **ph)
        history.append(rec)
        log(json.dumps(rec))
    loop_s = time.perf_counter() - t_loop
    sur.close()
    return dict(generations=generations, generations_per_s=generations / loop_s, loop_s=loop_s, setup_s=setup_s,
                history=history)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--generations", type=int, default=8)
    ap.add_argument("--mu", type=int, default=4096)
    ap.add_argument("--lam", type=int, default=4096)
    ap.add_argument("--screen", type=int, default=8)
    ap.add_argument("--T", type=int, default=5000)
    ap.add_argument("--tune", type=int, default=1)
    ap.add_argument("--pretrain", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed", type=int, default=2025)
    a = ap.parse_args()
    out = run(a.generations, a.mu, a.lam, a.screen, a.T, a.tune, a.pretrain, a.epochs, a.seed,
              log=lambda m: print(m, file=sys.stderr, flush=True))
    out.pop("history")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
