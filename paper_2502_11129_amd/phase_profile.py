"""Per-phase cycle counts of the rollout kernels: a profiling tool beside the
library, never on the simulation path.

`build` copies the kernel sources into DIR and instruments the copy: each
phase of a simulation step (forward kinematics and corner contacts; backward
pass and joint-space inertia; inverse; control and free velocity; contact
rows; projected Gauss-Seidel; integration) is bracketed by reads of the
shader clock (s_memtime), summed per wave over the launch and added into a
device array of the kernel's translation unit, with the wave count; the
tree-sparse kernel's inverse is split further (factor, clearing X, the
factor's first six rows, L^T y, L x = y, store).  The copy is compiled into
DIR/libsim.so.  `run` loads that library, rolls out the random-tree
population (8192 variants unless told otherwise) with the given options and
prints, per kernel translation unit and DoF capacity, the cycles per
wave-step of every phase.  The instrumentation adds a few instructions per
phase and keeps the kernels' registers within a few of the plain build.

    python -m paper_2502_11129_amd.phase_profile build --dir _phase
    python -m paper_2502_11129_amd.phase_profile run --dir _phase --steps 1000 --options '{"min_body_slots": 32}'
"""
from __future__ import annotations

import argparse
import json
import os
import shutil
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
PHASES = ("fk+corners", "backward+crba", "inverse", "control+vfree", "contact rows", "pgs", "integrate")
TREE_SUB = ("factor", "clear X", "first six rows", "L^T y", "L x = y", "store")
PGS_SUB = ("clamp rows", "contacts in registers", "overflow contacts")
# the first line of each phase (a comment that opens a ruled block, except
# the inverse, which opens with the factorisation's compile-time branch)
_MARKS = ("    // 1. forward kinematics", "    // 2. backward sweep", "    if constexpr (TREE) {",
          "    // 4. control and free", "    // 5. contact rows", "    // 6. projected Gauss", "    // 7. semi-implicit")


def _clock(acc, k, first=False):
    return ("{ const unsigned long long _t = __builtin_amdgcn_s_memtime(); "
            + ("" if first else f"{acc}[{k}] += _t - {acc}_p; ") + f"{acc}_p = _t; }}")


def instrument(src: str) -> str:
    """The kernel header with phase clocks (fails loudly if a mark is gone)."""
    out = []
    lines = src.split("\n")
    for line in lines:
        for k, m in enumerate(_MARKS):
            if line.startswith(m):
                rule = out.pop() if k != 2 else None    # ruled blocks: clock before the rule
                out.append("    " + _clock("_ph", k - 1, first=(k == 0)))
                if rule is not None:
                    out.append(rule)
        if line.strip() == "kstep += 1;":
            out.append("    " + _clock("_ph", 6))
        if line.startswith("  for (int it = 0; it < a.n_steps; ++it) {"):
            out.append("  unsigned long long _ph[7] = {0, 0, 0, 0, 0, 0, 0}, _ph_p = 0;")
            out.append("  unsigned long long _sub[6] = {0, 0, 0, 0, 0, 0}, _sub_p = 0;")
            out.append("  unsigned long long _pgs[3] = {0, 0, 0}, _pgs_p = 0;")
        if line.startswith("  // ---- write back ----"):
            out.append("  if (threadIdx.x == 0) { const int _b = NVC / 4; atomicAdd(&g_phase[_b][7], 1ull);")
            out.append("    for (int _i = 0; _i < 7; ++_i) atomicAdd(&g_phase[_b][_i], _ph[_i]);")
            out.append("    if (TREE) for (int _i = 0; _i < 6; ++_i) atomicAdd(&g_phase[16][_i], _sub[_i]);")
            out.append("    for (int _i = 0; _i < 3; ++_i) atomicAdd(&g_phase[8 + _b][_i], _pgs[_i]); }")
        out.append(line)
    s = "\n".join(out)
    s = s.replace("namespace simk {", "namespace simk {\nstatic __device__ unsigned long long g_phase[24][8];", 1)
    if s.count("s_memtime") != 8:
        raise RuntimeError("phase marks not found in the kernel source")
    # projected Gauss-Seidel: clamp rows, contacts in registers, overflow
    # contacts, summed over the sweeps
    pgs = ("      // (i) actuator clamp rows in hinge order.", "      // (ii) contact rows in (body, corner) order",
           "      for (int c = NCR; c < nc; ++c) {\n        const float* rows = ovf_rows")
    for k, anchor in enumerate(pgs):
        if s.count(anchor) != 1:
            raise RuntimeError(f"projected Gauss-Seidel mark {k} not found")
        s = s.replace(anchor, "      " + _clock("_pgs", k - 1, first=(k == 0)) + "\n" + anchor)
    # the overflow part ends with each sweep (the clamp rows' clock restarts
    # the next one), so its clock goes at the end of the sweep loop's body
    end = "        sd[7] = lam[0]; sd[8] = lam[1]; sd[9] = lam[2];\n      }\n    }\n"
    if s.count(end) != 1:
        raise RuntimeError("end of the projected Gauss-Seidel sweep not found")
    s = s.replace(end, end[:-len("    }\n")] + "      " + _clock("_pgs", 2) + "\n    }\n", 1)
    subs = ("#pragma unroll 1\n      for (int k = nv - 1; k >= 0; --k) {\n        const unsigned ak",
            "#pragma unroll\n      for (int s = 0; s < S; ++s) {\n        const int d = lane + 16 * s;\n        if (d < NVC) {\n"
            "#pragma unroll\n          for (int j = 0; j < NVC; ++j) sh.X[d * MST + j]",
            "      // the factor's first six rows", "      // L^T y = e_c", "      // L x = y over the DoFs",
            "      // registers and X hold the inverse negated")
    for k, anchor in enumerate(subs):
        if s.count(anchor) != 1:
            raise RuntimeError(f"tree-sparse sub-phase mark {k} not found")
        s = s.replace(anchor, "      " + _clock("_sub", k - 1, first=(k == 0)) + "\n" + anchor)
    end = "    } else {\n      // =====================================================================\n      // 3. inverse by"
    if s.count(end) != 1:
        raise RuntimeError("end of the tree-sparse inverse not found")
    return s.replace(end, "      " + _clock("_sub", 5) + "\n" + end)


def build(dirname: str) -> str:
    from . import build as B
    csrc = os.path.join(os.path.abspath(dirname), "csrc")
    if os.path.exists(csrc):
        shutil.rmtree(csrc)
    shutil.copytree(B.CSRC, csrc)
    hdr = os.path.join(csrc, "rollout_kernel.hpp")
    with open(hdr) as f:
        s = instrument(f.read())
    with open(hdr, "w") as f:
        f.write(s)
    # one read routine per kernel translation unit (no relocatable device code)
    inc = os.path.join(csrc, "rollout_inst.inc")
    with open(inc) as f:
        t = f.read()
    t += """
#ifdef PHASE_TU
#define PH_CAT2(a, b) a##b
#define PH_CAT(a, b) PH_CAT2(a, b)
extern "C" int PH_CAT(simk_phase_read_, PHASE_TU)(unsigned long long* out, int clear) {
  if (hipMemcpyFromSymbol(out, HIP_SYMBOL(simk::g_phase), sizeof(unsigned long long) * 192) != hipSuccess) return -1;
  if (clear) {
    static unsigned long long z[192];
    if (hipMemcpyToSymbol(HIP_SYMBOL(simk::g_phase), z, sizeof(z)) != hipSuccess) return -2;
  }
  return 0;
}
#endif
"""
    with open(inc, "w") as f:
        f.write(t)
    for tu in units(csrc):
        q = os.path.join(csrc, "kernels", f"rollout_{tu}.hip")
        with open(q) as f:
            body = f.read()
        with open(q, "w") as f:
            f.write(f"#define PHASE_TU {tu}\n" + body)
    return B.build(csrc=csrc, lib=os.path.join(os.path.abspath(dirname), "libsim.so"),
                   objdir=os.path.join(os.path.abspath(dirname), "obj"))


def units(csrc: str):
    """Kernel translation units that instantiate the per-bin rollout kernels
    (the single-launch kernel's unit has no read routine and is not profiled)."""
    kd = os.path.join(csrc, "kernels")
    out = []
    for f in sorted(os.listdir(kd)):
        if f.startswith("rollout_") and f.endswith(".hip"):
            with open(os.path.join(kd, f)) as fh:
                if "rollout_inst.inc" in fh.read():
                    out.append(f[len("rollout_"):-4])
    return out


def run(dirname: str, options: dict, steps: int, n: int = 8192, say=print):
    """Per-phase cycles per wave-step: list of dicts (unit, nvc, waves, phases, [sub-phases])."""
    import ctypes as C

    import numpy as np
    import torch

    from . import sim as S
    from . import workloads as W
    S._LIB_PATH = os.path.join(os.path.abspath(dirname), "libsim.so")
    lib = S.load()
    opts = {k: ({int(a): b for a, b in v.items()} if k == "ncr_by_nvc" else v) for k, v in options.items()}
    pop = W.random_trees(n)
    sim = S.Simulator(pop, **opts)
    tus = units(os.path.join(os.path.abspath(dirname), "csrc"))
    buf = (C.c_ulonglong * 192)()
    for tu in tus:
        getattr(lib, f"simk_phase_read_{tu}")(buf, 1)
    sim.rollout(steps)
    torch.cuda.synchronize()
    say(f"bins {sim.bins()} factorisation {sim.bin_factorization()}")
    rows = []
    for tu in tus:
        if getattr(lib, f"simk_phase_read_{tu}")(buf, 1) != 0:
            raise RuntimeError(f"phase read failed for {tu}")
        a = np.array(buf[:], dtype=np.float64).reshape(24, 8)
        for b in range(8):
            if a[b, 7] > 0:
                per = a[b, :7] / (a[b, 7] * steps)
                row = dict(unit=tu, nvc=4 * b, waves=int(a[b, 7]), phases=dict(zip(PHASES, per.tolist())),
                           total=float(per.sum()))
                if a[16, :6].any():
                    row["tree_sub"] = dict(zip(TREE_SUB, (a[16, :6] / (a[b, 7] * steps)).tolist()))
                row["pgs_sub"] = dict(zip(PGS_SUB, (a[8 + b, :3] / (a[b, 7] * steps)).tolist()))
                rows.append(row)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("what", choices=("build", "run"))
    ap.add_argument("--dir", default="_phase")
    ap.add_argument("--options", default="{}", help="sim_options fields as JSON")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--variants", type=int, default=8192)
    a = ap.parse_args(argv)
    if a.what == "build":
        print(build(a.dir), flush=True)
        return 0
    rows = run(a.dir, json.loads(a.options), a.steps, a.variants, say=lambda m: print(m, flush=True))
    print(f"{'unit':>8} {'nvc':>4} {'waves':>6} " + " ".join(f"{p:>14}" for p in PHASES) + f" {'total':>8}")
    for r in rows:
        print(f"{r['unit']:>8} {r['nvc']:>4} {r['waves']:>6} " +
              " ".join(f"{r['phases'][p]:>14.0f}" for p in PHASES) + f" {r['total']:>8.0f}")
        if "tree_sub" in r:
            print("         inverse sub-phases: " + ", ".join(f"{k} {v:.0f}" for k, v in r["tree_sub"].items()))
        print("         projected Gauss-Seidel: " + ", ".join(f"{k} {v:.0f}" for k, v in r["pgs_sub"].items()))
    print(json.dumps(rows), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
