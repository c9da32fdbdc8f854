"""Autotuner of the launch and packing options (sim_options).

The layout options never change results (same arithmetic in every layout);
they change how the population is cut into DoF bins and launched: contacts
kept in registers per DoF capacity, body capacity (merging bins), steps per
launch and the number of concurrent streams.  One option changes rounding
only: the kernels' factorisation of M~ (dense sweep or tree-sparse L^T L,
where a tree-sparse kernel of the bin's shape is compiled).  The tuner times short pilot rollouts
of the actual population (HIP events on the stream) and keeps the fastest
setting of one option at a time (coordinate descent, fixed order), so the
search costs a few dozen pilots.

`autotune_host` picks the host worker's factorisation of the joint-space
system (dense Cholesky or the tree-sparse L^T L; equal up to rounding) by
timing host rollouts of a sample of the population with each.
"""
from __future__ import annotations

import json
import os

from . import sim as S


def _time_rollout(pop, T, reps, **opts):
    import torch
    sim = S.Simulator(pop, **opts)
    st = torch.cuda.current_stream()
    sim.rollout(min(T, 250))                        # warm-up (first launches, caches)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        sim.rollout(T)
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    bins = sim.bins()
    sim.close()
    return best, bins


def _duel(cands, time_fn, rounds=3):
    """Times every candidate `rounds` times, interleaved so that drift of the
    GPU's clocks or temperature hits all of them alike; returns the index of
    the lowest median time and the medians."""
    import numpy as np
    times = [[] for _ in cands]
    for _ in range(rounds):
        for i, o in enumerate(cands):
            times[i].append(time_fn(o))
    med = [float(np.median(t)) for t in times]
    return int(np.argmin(med)), med


def candidates_ncr(nvc, ball=False, self_collision=False):
    """Compiled contact-register budgets for a DoF capacity (any body capacity)."""
    return sorted({k[2] for k in S.kernel_variants(ball, self_collision) if k[0] == nvc})


def autotune(pop, T_pilot=1000, reps=3, log=None, cache=None, min_gain=0.01, duel_margin=0.02, duel_max=4):
    """Returns (best options dict, list of trial records).  A setting is kept
    only when its pilot (best of `reps` rollouts) beats the current best by
    more than `min_gain`.  The pilots' noise is of the order of 1-2 %, so at
    the end the option sets whose pilots came within `duel_margin` of the
    best (at most `duel_max` of them) are timed again, interleaved, and the
    lowest median wins.  `cache`: optional JSON file path keyed by the
    population's DoF/body signature."""
    import numpy as np
    key = None
    if cache:
        nv = np.asarray(pop.nv)
        nb = np.asarray(pop.n_bodies)
        key = f"{pop.name}:{pop.n_variants}:{np.bincount(nv).tolist()}:{np.bincount(nb).tolist()}:{T_pilot}"
        if os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
            if key in store:
                return store[key]["options"], store[key]["trials"]
    trials = []

    def run(opts):
        t, bins = _time_rollout(pop, T_pilot, reps, **opts)
        trials.append(dict(options=dict(opts), seconds=t, bins=bins))
        if log:
            log(f"autotune {opts}: {t * 1e3:.2f} ms, bins {[(b[0], b[1], b[2], b[3]) for b in bins]}")
        return t

    def descend(best, best_t):
        """Coordinate descent from a starting point: single launch, streams,
        launch length, hipGraph replay of the rollout's launches, the
        contact budget of each DoF capacity present, then the tree-sparse
        factorisation."""
        special = getattr(pop, "ball", None) is not None or bool(getattr(pop, "self_collision", False))
        single = [] if special else [True]   # the multi-bin kernel has no ball or self-collision families
        for name, values in (("single_launch", single), ("streams", [4, 2, 1]), ("steps_per_launch", [250, 500]),
                             ("use_graph", [True])):
            for v in values:
                cand = dict(best, **{name: v})
                if cand.get("single_launch") and name == "streams":
                    continue                       # one launch uses one stream
                try:
                    t = run(cand)
                except S.SimError:
                    continue                       # e.g. a bin outside the single-launch kernel
                if t < best_t * (1.0 - min_gain):            # keep only clear wins
                    best, best_t = cand, t
        probe = S.Handle(pop, **best)
        nvcs = sorted({b[0] for b in probe.bins()})
        probe.close()
        for nvc in nvcs:
            for ncr in candidates_ncr(nvc, getattr(pop, "ball", None) is not None,
                                      bool(getattr(pop, "self_collision", False))):
                if ncr == best["ncr_by_nvc"].get(nvc):
                    continue
                cand = dict(best, ncr_by_nvc={**best["ncr_by_nvc"], nvc: ncr})
                try:
                    t = run(cand)
                except S.SimError:
                    continue                      # no kernel with that budget for this body capacity
                if t < best_t * (1.0 - min_gain):
                    best, best_t = cand, t
        # the tree-sparse factorisation, if some bin of this layout has it
        cand = dict(best, gpu_factorization="tree")
        probe = S.Handle(pop, **cand)
        has_tree = "tree" in probe.bin_factorization()
        probe.close()
        if has_tree:
            t = run(cand)
            if t < best_t * (1.0 - min_gain):
                best, best_t = cand, t
        return best, best_t

    # starting points: smallest body capacity per variant (more bins, some
    # kernels with fewer registers), every variant in 32-body kernels (fewer
    # bins), 32-body kernels only from 20 DoFs on with the smaller variants
    # merged into one 16-DoF, 16-body bin (whose kernels run two waves per
    # SIMD), and the same with the 20-DoF variants in 16-body kernels with 4
    # contacts in registers (also two waves per SIMD); a start that gives the
    # same bins as an earlier one is skipped
    results, seen = [], []
    for extra in (dict(min_body_slots=0), dict(min_body_slots=32),
                  dict(min_body_slots=32, slots32_min_nvc=20, min_nv_capacity=16),
                  dict(min_body_slots=32, slots32_min_nvc=24, min_nv_capacity=16, ncr_by_nvc={16: 8, 20: 4})):
        start_opts = dict(dict(streams=0, steps_per_launch=0, ncr_by_nvc={}), **extra)
        probe = S.Handle(pop, **start_opts)
        layout = sorted(tuple(b[:4]) for b in probe.bins())
        probe.close()
        if layout in seen:
            continue
        seen.append(layout)
        results.append(descend(start_opts, run(start_opts)))
    best, best_t = min(results, key=lambda r: r[1])
    close = []
    for tr in sorted(trials, key=lambda r: r["seconds"]):
        if tr["seconds"] <= best_t * (1.0 + duel_margin) and tr["options"] not in close:
            close.append(tr["options"])
    close = close[:duel_max]
    if len(close) > 1:
        def time_fn(o):
            t, bins = _time_rollout(pop, T_pilot, 2, **o)
            trials.append(dict(options=dict(o), seconds=t, bins=bins, final=True))
            return t
        i, med = _duel(close, time_fn)
        if log:
            log(f"autotune final round: medians {[round(m * 1e3, 2) for m in med]} ms, keeping {close[i]}")
        best = close[i]
    if cache:
        store = {}
        if os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
        store[key] = dict(options=best, trials=trials)
        with open(cache, "w") as f:
            json.dump(store, f)
    return best, trials


def autotune_host(pop, T_pilot=1000, threads=1, sample=64, log=None):
    """Faster host factorisation ("dense" or "tree") for this population:
    host rollouts of every k-th variant (about `sample` of them, so the mix of
    sizes is kept) over T_pilot steps with each; returns (name, {name: s})."""
    import numpy as np
    n = pop.n_variants
    idx = np.arange(0, n, max(1, n // max(1, sample)))
    sub = pop.subset(idx) if len(idx) < n else pop
    times = {}
    for f in S.HOST_FACTORIZATIONS:
        h = S.Handle(sub, host_factorization=f)
        _, sec = h.rollout_host(T_pilot, threads)
        h.close()
        times[f] = sec
        if log:
            log(f"autotune host {f}: {sec * 1e3:.1f} ms for {len(idx)} variants x {T_pilot} steps")
    return min(times, key=times.get), times
