#!/usr/bin/env python3
"""Benchmark: batched rollouts of the uneven-morphology population on one MI355X.

One bench step = one sim_rollout of the whole population (every variant,
T simulation steps: kinematics, dynamics, inverse, contacts, solver,
integration, fitness) with the model already resident in HBM.
Prints ONE JSON line (see the contract in the design doc).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3      # published MI355X FP32 vector peak (packed issue)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="trees", choices=["trees", "box_and_ball", "quadrupeds"],
                    help="trees: the uneven-morphology population (default); box_and_ball: a free box "
                         "and a free ball per variant (the paper's box-and-ball scene); quadrupeds: core + "
                         "four 5-brick limbs")
    ap.add_argument("--self-collision", action="store_true",
                    help="contacts between the boxes of one robot (quadrupeds workload)")
    ap.add_argument("--variants", type=int, default=None,
                    help="default 8192 (trees) / 512000 (box_and_ball) / 32768 (quadrupeds)")
    ap.add_argument("--horizon", type=int, default=None, help="default 5000 (trees) / 1000 (others)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="default launch options instead of the autotuned ones")
    ap.add_argument("--options", default=None,
                    help="launch options as JSON (sim_options fields); skips the autotuner")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates profiler byte counters)")
    ap.add_argument("--cpu-sample-steps", type=int, default=4000)
    ap.add_argument("--no-peak-probe", action="store_true",
                    help="skip the microbenchmarks that measure the attainable FP32, BF16 MFMA and copy peaks")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="instead of the GPU benchmark: the FP64 oracle over the whole snake (16 x 1000), box "
                         "(4096 x 2000), random-tree (8192 x 5000) and quadruped (32768 x 1000) populations on "
                         "this host's cores, all-core and single-thread rates, one JSON line")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-screened generation (200k labels, 1M pool) reported beside the "
                         "rollout throughput")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pop_full, sample_steps, workload="trees"):
    """The FP64 oracle, compiled -O3 -march=native on this host, over a
    bounded sample of the same workload: every 8th tree (1024 of the 8192),
    the first 16384 box-and-ball variants, or the first 64 quadrupeds, for
    sample_steps steps on all host threads (at most 16, the host share of
    one GPU); then one thread on the first 1/16 of that sample for a quarter
    of the steps (single-thread rate)."""
    import tempfile
    from oracle import oracle as O
    from paper_2502_11129_amd import workloads as W
    if workload == "box_and_ball":
        pop = W.box_and_ball(16384)
    elif workload == "quadrupeds":
        import dataclasses
        pop = dataclasses.replace(W.quadrupeds(64), self_collision=pop_full.self_collision)
    else:
        pop = W.random_trees(indices=range(0, pop_full.n_variants, 8))
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(16, avail))
    t0 = time.perf_counter()
    lib = O.load_native(os.path.join(tempfile.gettempdir(), f"oracle_native_{os.getpid()}"))
    t_build = time.perf_counter() - t0
    o = O.Oracle(pop, lib=lib)
    t0 = time.perf_counter()
    o.rollout(sample_steps, threads=cores)
    dt = time.perf_counter() - t0
    one = pop.subset(np.arange(0, pop.n_variants, 16))
    steps1 = max(1, sample_steps // 4)
    o1 = O.Oracle(one, lib=lib)
    t0 = time.perf_counter()
    o1.rollout(steps1, threads=1)
    dt1 = time.perf_counter() - t0
    what = "first" if workload in ("box_and_ball", "quadrupeds") else "every 8th"
    return {"value": pop.n_variants * sample_steps / dt, "unit": "variant-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{pop.n_variants} {what} variants x {sample_steps} steps, FP64, {cores} threads, "
                      f"{dt:.2f} s; single thread: {one.n_variants} of them x {steps1} steps, {dt1:.2f} s",
            "single_thread_value": one.n_variants * steps1 / dt1,
            "cpu_model": _cpu_model(), "host_threads_available": avail,
            "build": f"g++ -O3 -march=native on this host ({t_build:.1f} s, outside the timing)"}


def recorded_traffic(kernel, steps_per_launch):
    """HBM bytes per launch of `kernel` from the committed profiler counters,
    scaled by the copy calibration; None when the kernel source or the launch
    length differs from what was profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "rollout_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, rec["kernel_source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["kernel_source_sha256"]:
            return None
    table = rec["per_launch_kib_by_steps_per_launch"].get(str(steps_per_launch), {})
    if kernel not in table:
        return None
    fetch, write = table[kernel]
    return (fetch * rec["scale"]["FETCH_SIZE"] + write * rec["scale"]["WRITE_SIZE"]) * 1024.0


def cpu_configs():
    """The FP64 oracle (-O3 -march=native on this host) over every population of
    the benchmark configurations, whole, on all host threads (at most 16, the
    host share of one GPU), and on one thread over a sample of each."""
    import tempfile
    from oracle import oracle as O
    from paper_2502_11129_amd import workloads as W
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(16, avail))
    lib = O.load_native(os.path.join(tempfile.gettempdir(), f"oracle_native_{os.getpid()}"))
    rows = []
    for name, pop, T in (("snakes", W.snake(16), 1000), ("boxes", W.boxes(4096), 2000),
                         ("random trees", W.random_trees(8192), 5000), ("quadrupeds", W.quadrupeds(32768), 1000)):
        o = O.Oracle(pop, lib=lib)
        t0 = time.perf_counter()
        o.rollout(T, threads=cores)
        dt = time.perf_counter() - t0
        one = pop.subset(np.arange(0, pop.n_variants, max(1, pop.n_variants // 64)))
        T1 = max(1, T // 4)
        o1 = O.Oracle(one, lib=lib)
        t0 = time.perf_counter()
        o1.rollout(T1, threads=1)
        dt1 = time.perf_counter() - t0
        rows.append({"workload": name, "variants": pop.n_variants, "steps": T, "seconds": dt,
                     "variant_steps_per_s": pop.n_variants * T / dt, "threads": cores,
                     "single_thread_variant_steps_per_s": one.n_variants * T1 / dt1,
                     "single_thread_sample": f"{one.n_variants} variants x {T1} steps"})
        print(f"{name}: {pop.n_variants} x {T} in {dt:.1f} s on {cores} threads", file=sys.stderr, flush=True)
    print(json.dumps({"kind": "oracle", "unit": "variant-steps/s", "cpu_model": _cpu_model(),
                      "host_threads_available": avail, "configs": rows}), flush=True)


def main():
    args = parse()
    if args.cpu_configs:
        cpu_configs()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "variants are independent, so more GPUs would each take a contiguous DoF-balanced share.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2502_11129_amd import workloads as W
    from paper_2502_11129_amd.flops import flops_per_variant, bytes_per_rollout
    from paper_2502_11129_amd.sim import Simulator

    if args.workload == "box_and_ball":
        pop = W.box_and_ball(args.variants or 512000)
        T = args.horizon or 1000
        wname = (f"box-and-ball (a free box and a free ball per variant), {pop.n_variants} variants x {T} steps, "
                 "dt=0.002, K=8")
    elif args.workload == "quadrupeds":
        import dataclasses
        T = args.horizon or 1000
        pop = dataclasses.replace(W.quadrupeds(args.variants or 32768, steps=T), self_collision=args.self_collision)
        wname = (f"quadrupeds (core + four 5-brick limbs){' with self-collision' if args.self_collision else ''}, "
                 f"{pop.n_variants} variants x {T} steps, dt=0.002, K=8")
    else:
        pop = W.random_trees(args.variants or 8192)
        T = args.horizon or 5000
        wname = (f"uneven-morphology random trees (4-20 hinges, depth<=4), "
                 f"{pop.n_variants} variants x {T} steps, dt=0.002, K=8")
    options, trials = {}, []
    if args.options:
        options = {k: ({int(a): b for a, b in v.items()} if k == "ncr_by_nvc" else v)
                   for k, v in json.loads(args.options).items()}
    elif not args.no_autotune:
        from paper_2502_11129_amd.autotune import autotune
        # pilots over the whole horizon: the first steps of a dropped population
        # (free fall, few contacts) rank the launch options differently
        options, trials = autotune(pop, T_pilot=T, log=lambda m: print(m, file=sys.stderr, flush=True))
    # per-bin launch timing (HIP events around each bin's launches) cannot be
    # recorded inside a captured graph: a graph-replayed run is timed as is and
    # the per-kernel figures come from one more rollout of the same layout
    # launched eagerly
    graph = bool(options.get("use_graph"))
    sim = Simulator(pop, time_launches=not graph, **options)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        sim.rollout(T)
    torch.cuda.synchronize()
    # one event between consecutive rollouts (recording adds no host sync):
    # the whole span gives the value, the single rollouts its spread
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        sim.rollout(T)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = evs[0].elapsed_time(evs[-1])
    rollout_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    ms_per_step = gpu_ms / args.steps
    vsteps = pop.n_variants * T
    value = vsteps * args.steps / (gpu_ms / 1e3)

    if args.copy_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if graph:
        sim_t = Simulator(pop, time_launches=True, **dict(options, use_graph=False))
        sim_t.rollout(T)
        torch.cuda.synchronize()
        times, vb, bins, facs = sim_t.launch_times(), sim_t.variant_bins(), sim_t.bins(), sim_t.bin_factorization()
        sim_t.close()
    else:
        times, vb, bins, facs = sim.launch_times(), sim.variant_bins(), sim.bins(), sim.bin_factorization()
    rows_contact, rows_clamp, status = sim.counters()
    fl_var = flops_per_variant(pop, T, rows_contact, rows_clamp,
                               factorization=np.array([facs[b] for b in vb]))
    fl = fl_var.sum()
    # dominant kernel: the bin whose launches took longest in the last rollout
    # (HIP events around its launches on its own stream)
    dom = int(np.argmax([t[0] for t in times]))
    dom_ms, dom_launches = times[dom]
    per_launch_s = dom_ms / 1e3 / max(dom_launches, 1)
    dom_flops_per_launch = fl_var[vb == dom].sum() / max(dom_launches, 1)
    achieved = dom_flops_per_launch / per_launch_s / 1e12
    all_bins = fl / (ms_per_step / 1e3) / 1e12
    byt = bytes_per_rollout(pop)
    nvc, nbody, ncr, nvar = bins[dom]
    ball = "true" if getattr(pop, "ball", None) is not None else "false"
    selfc = "true" if getattr(pop, "self_collision", False) else "false"
    tree = "true" if facs[dom] == "tree" else "false"
    kernel_name = f"rollout_kernel<{nvc}, {nbody // 16}, {ncr}, {ball}, {selfc}, {tree}>"
    if options.get("single_launch"):
        # one kernel runs every bin: its launches carry the whole rollout
        kernel_name = "rollout_multi_kernel"
        nvar = pop.n_variants
        dom_flops_per_launch = fl / max(dom_launches, 1)
        achieved = dom_flops_per_launch / per_launch_s / 1e12
    traffic = recorded_traffic(kernel_name, options.get("steps_per_launch") or 1000)

    out = {
        "metric": "variant-steps/sec at 1 MI355X",
        "value": value,
        "unit": "variant-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname,
                   "variants": pop.n_variants, "horizon": T, "bins": bins,
                   "frozen_variants": int((status != 0).sum()),
                   "mean_contacts_per_step": float(rows_contact.sum() / (pop.n_variants * T)),
                   "options": options, "autotune_trials": len(trials),
                   "wall_s": wall},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": kernel_name,
                     "kernel_variants": nvar, "kernel_launches_per_step": dom_launches,
                     "kernel_avg_launch_ms": per_launch_s * 1e3,
                     "kernel_flops_per_launch": dom_flops_per_launch,
                     "all_bins_achieved": all_bins, "all_bins_frac": all_bins / FP32_VECTOR_PEAK_TFLOPS,
                     "bin_ms_per_step": [round(t[0], 3) for t in times],
                     "flops_per_step": fl, "hbm_bytes_per_step": byt,
                     "hbm_GBs": byt / (ms_per_step / 1e3) / 1e9},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pop, args.cpu_sample_steps, args.workload)
    if not args.no_surrogate:
        # the learned part's metric: surrogate-screened candidates/s at its measured
        # top-5 % recall, against plain simulation, on the same simulator
        from paper_2502_11129_amd.screening import run as screening_run
        sr = screening_run(log=lambda m: print(m, file=sys.stderr, flush=True))
        out["surrogate"] = {
            "metric": "surrogate-screened candidates/sec @ top-5% recall",
            "screened_candidates_per_s": sr["screened_candidates_per_s"],
            "plain_candidates_per_s": sr["plain_candidates_per_s"],
            "speedup_vs_plain": sr["speedup_vs_plain"],
            "holdout_recall_top5": sr["holdout_recall_top5"], "holdout_spearman": sr["holdout_spearman"],
            "holdout_recall_ceiling": sr["holdout_recall_ceiling"],
            "target": {"speedup": 5.0, "recall": 0.9},
            "config": {k: sr[k] for k in ("n_train", "n_holdout", "pool", "keep_frac", "T", "epochs", "batch")},
            "equal_gpu_time": sr["equal_time"],
            "detail": {k: v for k, v in sr.items() if k.endswith("_s") or k.startswith(("kept", "unscreened"))},
        }
    out["rollouts"] = rollout_spread(rollout_ms, pop.n_variants * T)
    if not args.no_peak_probe:
        # attainable peaks of this GPU (after the timed region), beside the published ones
        from paper_2502_11129_amd import probe
        peaks = probe.all_peaks()
        out["peak_probe"] = peaks
        out["roofline"]["peak_measured"] = peaks["fp32_fma_tflops"]
        out["roofline"]["frac_of_measured"] = achieved / peaks["fp32_fma_tflops"]
        out["roofline"]["all_bins_frac_of_measured"] = all_bins / peaks["fp32_fma_tflops"]
    print(json.dumps(out), flush=True)


def rollout_spread(ms, vsteps):
    """Per-rollout times of the timed region, the median throughput and a 95 %
    confidence interval of the mean throughput (Student t over the rollouts)."""
    v = np.asarray([vsteps / (m / 1e3) for m in ms], np.float64)
    rec = {"ms": [round(m, 3) for m in ms], "median_value": float(np.median(v)), "ci95_value": None}
    if len(v) >= 2:
        from scipy.stats import t as student_t
        half = float(student_t.ppf(0.975, len(v) - 1) * v.std(ddof=1) / np.sqrt(len(v)))
        rec["ci95_value"] = [float(v.mean() - half), float(v.mean() + half)]
    return rec


if __name__ == "__main__":
    main()
