"""Surrogate-screened evaluation of candidate robots (one generation).

1. Label n_train random-tree genotypes with exact rollouts of T steps.
2. Train the surrogate on the standardised labels (Adam, batch 4096).
3. Judge its ranking on a held-out set simulated exactly: top-5 % recall and
   Spearman's rho.
4. Screen a pool of candidates: features -> predictions -> top fraction on
   the GPU, then simulate the kept candidates exactly (the simulator is the
   judge of every kept candidate).

Ablation at equal GPU time: the pool's first candidates simulated plainly
for as long as the screened pass took, best and top-1 % fitness of both.

Throughput compared: screened candidates per second,
  pool / (t_features + t_predict + t_topk + t_resim(kept)),
against plain simulation, candidates / t_sim(candidates), both from GPU event
times of the same simulator.  Host time to build robot models from genotypes
is reported separately (it is the same per simulated candidate in both).

Usage: python -m paper_2502_11129_amd.screening [--train 200000] [--pool 1000000] ...
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def spearman_rank(x, y):
    """Spearman's rho (Pearson correlation of average ranks), for reporting."""
    from scipy.stats import rankdata
    rx, ry = rankdata(x), rankdata(y)
    rx -= rx.mean()
    ry -= ry.mean()
    return float((rx * ry).sum() / np.sqrt((rx * rx).sum() * (ry * ry).sum()))


def recall_top(pred, true, frac):
    k = max(1, int(round(frac * len(true))))
    a = np.lexsort((np.arange(len(pred)), -pred))[:k]
    b = np.lexsort((np.arange(len(true)), -true))[:k]
    return len(np.intersect1d(a, b)) / k


def run(n_train=200000, n_hold=10000, pool=1000000, keep_frac=0.05, T=5000, epochs=30, batch=4096, seed=0,
        log=print):
    import torch
    from . import workloads as W
    from .surrogate import Surrogate, screen, simulate_fitness, train

    out = dict(n_train=n_train, n_holdout=n_hold, pool=pool, keep_frac=keep_frac, T=T, epochs=epochs, batch=batch)
    t0 = time.perf_counter()
    g_train = W.random_genotypes(n_train, key=100 + seed)
    y, sim_s, host_s = simulate_fitness(g_train, T=T)
    out["label_gpu_s"], out["label_host_s"] = sim_s, host_s
    out["plain_candidates_per_s"] = n_train / sim_s
    log(f"labelled {n_train} genotypes: GPU {sim_s:.2f} s, model building {host_s:.1f} s")

    s = Surrogate(params=W.mlp_init(seed), max_batch=batch)
    X = s.features(s.upload_genotypes(g_train))
    z, mu, sd = s.standardize(torch.from_numpy(y).cuda())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    losses = train(s, X, z, epochs=epochs, batch=batch, seed=seed)
    ev[1].record()
    torch.cuda.synchronize()
    out["train_gpu_s"] = ev[0].elapsed_time(ev[1]) / 1e3
    out["train_loss_first_last"] = [float(losses[0].mean()), float(losses[-1].mean())]
    log(f"trained {epochs} epochs in {out['train_gpu_s']:.2f} s: loss {losses[0].mean():.3f} -> {losses[-1].mean():.3f}")

    g_hold = W.random_genotypes(n_hold, key=200 + seed)
    y_hold, _, _ = simulate_fitness(g_hold, T=T)
    p_hold = s.predict(s.features(s.upload_genotypes(g_hold))).cpu().numpy()
    out["holdout_recall_top5"] = recall_top(p_hold, y_hold, 0.05)
    out["holdout_spearman"] = spearman_rank(p_hold, y_hold)
    # what any predictor can reach: the holdout simulated again from initial
    # positions one float32 ulp away, ranked against the first simulation
    y_nudged, _, _ = simulate_fitness(g_hold, T=T, nudge=seed + 1)
    out["holdout_recall_ceiling"] = recall_top(y_nudged, y_hold, 0.05)
    out["holdout_spearman_ceiling"] = spearman_rank(y_nudged, y_hold)
    log(f"holdout: top-5% recall {out['holdout_recall_top5']:.3f}, Spearman {out['holdout_spearman']:.3f} "
        f"(ceiling from a rerun one float32 ulp apart: {out['holdout_recall_ceiling']:.3f}, "
        f"{out['holdout_spearman_ceiling']:.4f})")

    g_pool = W.random_genotypes(pool, key=300 + seed)
    gd = s.upload_genotypes(g_pool)
    k = int(round(keep_frac * pool))
    screen(s, gd, pool, k)                              # warm-up of the screening kernels
    top, pred, st = screen(s, gd, pool, k)
    top = top.cpu().numpy()
    f_top, resim_s, resim_host_s = simulate_fitness(g_pool.take(top), T=T)
    out.update(st)
    out["resim_gpu_s"], out["resim_host_s"] = resim_s, resim_host_s
    t_screen = st["features_s"] + st["predict_s"] + st["topk_s"] + resim_s
    out["screened_candidates_per_s"] = pool / t_screen
    out["speedup_vs_plain"] = out["screened_candidates_per_s"] / out["plain_candidates_per_s"]
    # what the kept set is worth: compare with an unscreened sample of the same size
    f_rand, _, _ = simulate_fitness(g_pool.take(np.arange(k)), T=T)
    out["kept_mean_fitness"] = float(np.nanmean(f_top))
    out["unscreened_mean_fitness"] = float(np.nanmean(f_rand))
    out["kept_best_fitness"] = float(np.nanmax(f_top))
    out["unscreened_best_fitness"] = float(np.nanmax(f_rand))
    # ablation at equal GPU time: plain simulation of as many pool candidates
    # as fit in the screened pass's time, against the screened pass
    n_eq = min(pool, max(1, int(out["plain_candidates_per_s"] * t_screen)))
    f_eq, eq_s, _ = simulate_fitness(g_pool.take(np.arange(n_eq)), T=T)
    top_n = max(1, min(k, n_eq) // 100)
    out["equal_time"] = dict(
        plain_candidates=n_eq, plain_gpu_s=eq_s, screened_gpu_s=t_screen, top_n=top_n,
        screened_best=float(np.nanmax(f_top)), plain_best=float(np.nanmax(f_eq)),
        screened_top_mean=float(np.sort(f_top[np.isfinite(f_top)])[-top_n:].mean()),
        plain_top_mean=float(np.sort(f_eq[np.isfinite(f_eq)])[-top_n:].mean()))
    log(f"equal GPU time ({t_screen:.2f} s): screened best {out['equal_time']['screened_best']:.4f}, "
        f"top-{top_n} mean {out['equal_time']['screened_top_mean']:.4f}; plain ({n_eq} candidates) best "
        f"{out['equal_time']['plain_best']:.4f}, top-{top_n} mean {out['equal_time']['plain_top_mean']:.4f}")
    out["wall_s"] = time.perf_counter() - t0
    log(f"screened {pool} candidates, kept {k}: {out['screened_candidates_per_s']:.0f} candidates/s "
        f"vs plain {out['plain_candidates_per_s']:.0f} ({out['speedup_vs_plain']:.1f}x); mean fitness kept "
        f"{out['kept_mean_fitness']:.4f} vs unscreened {out['unscreened_mean_fitness']:.4f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200000)
    ap.add_argument("--holdout", type=int, default=10000)
    ap.add_argument("--pool", type=int, default=1000000)
    ap.add_argument("--keep", type=float, default=0.05)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    r = run(a.train, a.holdout, a.pool, a.keep, a.steps, a.epochs, seed=a.seed, log=lambda m: print(m, flush=True))
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
