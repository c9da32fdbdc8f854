"""The paper's combined CPU + GPU measurement (Sec. 6 "Results"), on this
simulator: for each population size N, Sequential GPU, Sequential CPU (host
threads), Naive Sum (their sum), Combined (wall clock of the concurrent run
whose split comes from a pilot run) and the GPU share.

Usage: python -m paper_2502_11129_amd.split_bench [--workload quadrupeds] [--steps 1000] [--sizes 32,128,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def measure(pop, T, threads, rule="makespan", pilot_T=None, host_sample=None, log=print, progress=None,
            host_factorization=None):
    """pilot_T: steps of the pilot runs (default the full horizon T, as the
    paper's initial benchmarking runs: a short pilot of a dropped scene sees
    only the free fall, where the host's per-step cost is lowest).
    host_factorization: "dense", "tree" or None (the faster on a sample)."""
    import torch
    say = progress or (lambda m: None)
    from .sim import Simulator
    if host_factorization is None:
        from .autotune import autotune_host
        host_factorization, _ = autotune_host(pop, pilot_T or T, threads, sample=max(threads * 2, 32))
    say(f"n={pop.n_variants}: host factorisation {host_factorization}")
    sim = Simulator(pop, host_factorization=host_factorization)
    n = pop.n_variants
    st = torch.cuda.current_stream()
    # sequential GPU (after a warm-up)
    sim.rollout(T)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    sim.rollout(T)
    e1.record(st)
    e1.synchronize()
    seq_gpu = time.perf_counter() - t0
    seq_gpu_events = e0.elapsed_time(e1) / 1e3
    say(f"n={n}: sequential GPU {seq_gpu:.3f} s")
    # sequential CPU: every variant on host threads
    _, seq_cpu = sim.rollout_host(T, threads)
    say(f"n={n}: sequential CPU {seq_cpu:.3f} s")
    # pilot and allocation
    plan = sim.plan_split(pilot_T or T, threads, host_sample or max(threads * 4, min(n, 256)))
    n_host = plan["n_host_makespan"] if rule == "makespan" else plan["n_host_paper"]
    say(f"n={n}: pilot split, {n_host} variants on the host")
    # combined run
    t = sim.rollout_split(T, n_host, threads)
    out = dict(n=n, T=T, threads=threads, rule=rule, seq_gpu_s=seq_gpu, seq_gpu_events_s=seq_gpu_events,
               seq_cpu_s=seq_cpu, naive_sum_s=seq_gpu + seq_cpu, combined_s=t["combined_s"],
               combined_gpu_s=t["gpu_s"], combined_host_s=t["host_s"], n_host=n_host,
               gpu_percent=100.0 * (n - n_host) / n, host_factorization=host_factorization, plan=plan)
    log(json.dumps(out))
    sim.close()
    return out


def main():
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="quadrupeds", choices=["quadrupeds", "trees", "boxes", "box_and_ball"])
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--sizes", default="32,128,512,2048,8192,32768")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--rule", default="makespan", choices=["makespan", "paper"])
    ap.add_argument("--host-factorization", default=None, choices=["dense", "tree"],
                    help="host worker's factorisation (default: the faster on a sample)")
    a = ap.parse_args()
    make = {"quadrupeds": lambda n: W.quadrupeds(n, steps=a.steps), "trees": W.random_trees, "boxes": W.boxes,
            "box_and_ball": lambda n: W.box_and_ball(n, steps=a.steps)}[a.workload]
    for n in (int(x) for x in a.sizes.split(",")):
        measure(make(n), a.steps, a.threads, a.rule, log=lambda m: print(m, flush=True),
                progress=lambda m: print(m, file=sys.stderr, flush=True), host_factorization=a.host_factorization)


if __name__ == "__main__":
    main()
