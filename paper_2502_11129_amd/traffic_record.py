"""Build the HBM traffic record that bench.py reports (profiles/rollout_traffic.json)
from rocprofv3 counter runs of bench.py.

Each run is one `rocprofv3 --pmc FETCH_SIZE` or `--pmc WRITE_SIZE` pass with
`-f csv` over `bench.py ... --options '{..., "steps_per_launch": L}'
--copy-probe`; the copy probe (one plain 1 GiB device-to-device copy in the
same process) calibrates each counter: scale = 1 GiB / what the counter reads
for the copy.  Per rollout kernel the record keeps the mean FETCH_SIZE and
WRITE_SIZE (KiB) of its launches after the first (the first is the zero-step
launch at bind time), keyed by the launch length L, with the SHA-256 of the
kernel source so that bench.py drops the figure once the kernel changes.

    python -m paper_2502_11129_amd.traffic_record --out profiles/rollout_traffic.json \\
        --run 1000:gpurun_out/traffic/f_A_1000:gpurun_out/traffic/w_A_1000 [--run ...]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = "paper_2502_11129_amd/csrc/rollout_kernel.hpp"
COPY_BYTES_KIB = 1 << 20          # the 1 GiB copy probe


def _kernel_key(name: str) -> str:
    m = re.search(r"(rollout_kernel<[^>]*>|rollout_multi_kernel)", name)
    return m.group(1) if m else name


def read_counter(run_dir: str, counter: str):
    """{kernel name: [value per dispatch in dispatch order]} of one pass."""
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    per = defaultdict(float)                 # (dispatch, kernel) -> summed value
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                per[(int(row["Dispatch_Id"]), row["Kernel_Name"])] += float(row["Counter_Value"])
    out = defaultdict(list)
    for (d, k), v in sorted(per.items()):
        out[k].append(v)
    return out


def calibration(values) -> float:
    """Scale of a counter: the copy probe's 1 GiB over its reading (the
    copy kernel is the non-rollout dispatch with the largest reading)."""
    best = 0.0
    for k, vs in values.items():
        if "rollout" in k:
            continue
        best = max(best, max(vs))
    if best <= 0:
        raise ValueError("copy probe not found in the counter run")
    return COPY_BYTES_KIB / best


def build(runs, out_path, workload):
    table, scales = {}, defaultdict(list)
    for L, fdir, wdir in runs:
        f, w = read_counter(fdir, "FETCH_SIZE"), read_counter(wdir, "WRITE_SIZE")
        scales["FETCH_SIZE"].append(calibration(f))
        scales["WRITE_SIZE"].append(calibration(w))
        t = table.setdefault(str(L), {})
        for name, fv in f.items():
            if "rollout_kernel<" not in name or name not in w or len(fv) < 2:
                continue
            wv = w[name]
            t[_kernel_key(name)] = [sum(fv[1:]) / len(fv[1:]), sum(wv[1:]) / len(wv[1:])]
    scale = {k: round(sum(v) / len(v), 3) for k, v in scales.items()}
    with open(os.path.join(ROOT, KERNEL_SOURCE), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    rec = {"kernel_source": KERNEL_SOURCE, "kernel_source_sha256": sha, "workload": workload,
           "scale": scale, "per_launch_kib_by_steps_per_launch": table,
           "calibration_runs": {k: [round(x, 4) for x in v] for k, v in scales.items()},
           "summary": "profiles/rollout_trees_8192x1000_counters.md"}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--run", action="append", required=True, help="L:fetch_dir:write_dir")
    ap.add_argument("--workload", default="8192 random trees, one 1000-step rollout per run, "
                                          "the packing layouts the autotuner chooses between")
    a = ap.parse_args(argv)
    runs = []
    for r in a.run:
        L, fd, wd = r.split(":")
        runs.append((int(L), fd, wd))
    rec = build(runs, a.out, a.workload)
    for L, t in rec["per_launch_kib_by_steps_per_launch"].items():
        for k, (fv, wv) in t.items():
            print(f"L={L} {k}: FETCH {fv:.1f} KiB, WRITE {wv:.1f} KiB", flush=True)
    print("scale", rec["scale"], flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
