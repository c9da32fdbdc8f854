"""Host-side pieces of bench.py: the spread of the timed rollouts, the lookup
of the recorded HBM traffic (kernel source hash, launch length and kernel
name must all match what was profiled) and the one-GPU guard."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_rollout_spread_median_and_interval():
    ms = [263.1, 264.0, 262.5, 263.7, 264.4]
    vsteps = 8192 * 5000
    r = bench.rollout_spread(ms, vsteps)
    v = np.array([vsteps / (m / 1e3) for m in ms])
    assert r["median_value"] == pytest.approx(np.median(v))
    lo, hi = r["ci95_value"]
    assert lo < v.mean() < hi
    # t(0.975, 4) = 2.776: the half width over the standard error
    assert (hi - lo) / 2 == pytest.approx(2.7764451 * v.std(ddof=1) / np.sqrt(5), rel=1e-6)
    assert bench.rollout_spread([250.0], vsteps)["ci95_value"] is None


def _record(tmp_path, sha, steps=1000):
    src = tmp_path / "kernel.hpp"
    src.write_text("// kernel source stand-in\n")
    (tmp_path / "profiles").mkdir()
    rec = {"kernel_source": "kernel.hpp", "kernel_source_sha256": sha, "scale": {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0},
           "per_launch_kib_by_steps_per_launch": {str(steps): {"rollout_kernel<24, 2, 8, false, false, false>": [100.0, 30.0]}}}
    (tmp_path / "profiles" / "rollout_traffic.json").write_text(json.dumps(rec))
    return hashlib.sha256(src.read_bytes()).hexdigest()


def test_recorded_traffic_scales_and_refuses_stale_records(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    good = _record(tmp_path, "0" * 64)
    assert bench.recorded_traffic("rollout_kernel<24, 2, 8, false, false, false>", 1000) is None   # source changed
    (tmp_path / "profiles" / "rollout_traffic.json").unlink()
    (tmp_path / "profiles").rmdir()
    _record(tmp_path, good)
    assert bench.recorded_traffic("rollout_kernel<24, 2, 8, false, false, false>", 1000) == (100.0 * 2.0 + 30.0) * 1024
    assert bench.recorded_traffic("rollout_kernel<24, 2, 8, false, false, false>", 250) is None    # other launch length
    assert bench.recorded_traffic("rollout_kernel<20, 2, 8, false, false, false>", 1000) is None   # kernel not profiled


def test_committed_traffic_record_names_profiled_kernels():
    with open(os.path.join(ROOT, "profiles", "rollout_traffic.json")) as f:
        rec = json.load(f)
    assert os.path.exists(os.path.join(ROOT, rec["kernel_source"]))
    assert rec["scale"]["FETCH_SIZE"] > 0 and rec["scale"]["WRITE_SIZE"] > 0
    for steps, table in rec["per_launch_kib_by_steps_per_launch"].items():
        assert int(steps) > 0
        assert all(k.startswith("rollout_kernel<") and len(v) == 2 for k, v in table.items())


def test_committed_traffic_record_matches_the_kernel_source():
    """The record is re-taken whenever the rollout kernel changes: a stale
    record would silently drop the bench line's traffic figure."""
    assert bench.recorded_traffic("rollout_kernel<24, 2, 8, false, false, false>", 1000) is not None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_autotune_final_round_takes_the_lowest_median_interleaved():
    from paper_2502_11129_amd.autotune import _duel
    script = {"a": iter([1.00, 1.10, 1.00]), "b": iter([0.99, 0.98, 1.30]), "c": iter([1.05, 0.90, 1.06])}
    calls = []

    def time_fn(o):
        calls.append(o)
        return next(script[o])

    i, med = _duel(["a", "b", "c"], time_fn)
    assert calls == ["a", "b", "c"] * 3          # interleaved rounds
    assert med == [1.00, 0.99, 1.05]
    assert i == 1
