"""Driver for the sanitizer tests (run in a subprocess that preloads the ASan
runtime): `oracle` runs the FP64 oracle built with ASan + UBSan over every
workload family; `sim <library>` runs the host side of a libsim.so built the
same way (validation and packing, host-worker rollouts with both
factorisations on several threads, chunk planning, the host-failure path).
Any sanitizer finding aborts the process."""
import dataclasses
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2502_11129_amd import workloads as W  # noqa: E402


def _cases():
    return [("snakes", W.snake(3), 200), ("trees", W.random_trees(8), 100),
            ("quadrupeds with self-collision", dataclasses.replace(W.quadrupeds(3), self_collision=True), 100),
            ("box-and-ball", W.box_and_ball(6), 150), ("crossing chains", W.twisted_chains(3), 80),
            ("boxes", W.boxes(8), 150)]


def run_oracle(workdir):
    from oracle import oracle as O
    lib = O.load_sanitized(workdir)
    for name, pop, T in _cases():
        o = O.Oracle(pop, lib=lib)
        o.step(T, 2)
        q, v, k, st = o.get_state()
        c = o.contacts(0, o.variant_state(0)[0], max_contacts=4096)
        R, p, _, _ = o.fk(0, o.variant_state(0)[0])
        a, b = o.counters()
        assert (k == T).all() and np.isfinite(q).all()
        print(f"{name}: {T} steps, {len(c['depth'])} contacts of variant 0", flush=True)


def run_sim(lib_path):
    from paper_2502_11129_amd import sim as S
    S._LIB_PATH = lib_path
    S.load()
    for name, pop, T in _cases():
        for fac in ("dense", "tree"):
            h = S.Handle(pop, host_factorization=fac, min_body_slots=32 if name == "trees" else 0)
            f, _ = h.rollout_host(T, threads=3)
            ends = h.chunk_plan(h.workspace_bytes() // 2 + 4096)
            h.bins(), h.bin_factorization(), h.variant_bins()
            h.close()
            assert np.isfinite(f).all() and ends[-1] == pop.n_variants
        print(f"{name}: host rollouts with both factorisations, chunk plan {ends}", flush=True)
    h = S.Handle(W.random_trees(40), host_fault_items=2)
    try:
        h.rollout_host(10, threads=4)
        raise AssertionError("the injected failures were not reported")
    except S.SimError as e:
        assert e.code == S.SIM_E_HOST
    for bad in (dict(min_nv_capacity=10), dict(host_fault_items=-1), dict(gpu_factorization="x")):
        try:
            S.Handle(W.snake(2), **bad)
        except (S.SimError, ValueError):
            pass
    print("failure and validation paths", flush=True)


if __name__ == "__main__":
    if sys.argv[1] == "oracle":
        run_oracle(sys.argv[2])
    else:
        run_sim(sys.argv[2])
    print("clean", flush=True)
