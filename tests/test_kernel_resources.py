"""Register budgets of the rollout kernels, from the compiler's resource
report of the last build (`_build/kernel_resources.json`, written by
build()): the families below 20 DoFs with at most 8 contacts in registers
fit 256 registers and run two waves per SIMD (holding the contacts' solver
scalars in registers, as the larger families do, would cost them that: the
box-and-ball kernel ran 39 % slower so); only the two-wave 20-DoF, 16-body
kernels with 2 or 4 contacts in registers spill, and by a bounded amount."""
import json
import os
import re

import pytest

from paper_2502_11129_amd import build as B

PATH = os.path.join(B.BUILD, B.RESOURCES)
PAT = re.compile(r"rollout_kernelILi(\d+)ELi(\d+)ELi(\d+)ELb([01])ELb([01])ELb([01])E")


def _kernels():
    if not os.path.exists(PATH):
        pytest.skip("no resource report: run build() first")
    with open(PATH) as f:
        rep = json.load(f)
    fams = {}
    for name, r in rep.items():
        m = PAT.search(name)
        if m:
            fams[tuple(int(x) for x in m.groups())] = r
    return rep, fams


def _two_wave_rule(nvc, sb, ncr):
    """The families the kernel source builds for two waves per SIMD."""
    return (sb == 1 and ncr <= 2 and nvc <= 20) or (sb == 1 and ncr == 4 and nvc == 20) or (ncr == 8 and nvc == 16)


def test_small_families_keep_two_waves_per_simd():
    _, fams = _kernels()
    assert len(fams) >= 30
    checked = 0
    for (nvc, sb, ncr, ball, self_, tree), r in fams.items():
        if _two_wave_rule(nvc, sb, ncr) or (nvc < 20 and ncr <= 8):
            assert r["Occupancy [waves/SIMD]"] >= 2, ((nvc, sb, ncr, ball, self_, tree), r)
            checked += 1
    assert checked >= 12


def test_only_the_two_wave_20_dof_kernels_spill():
    rep, fams = _kernels()
    for key, r in fams.items():
        scratch = r["ScratchSize [bytes/lane]"]
        if key[:3] in ((20, 1, 2), (20, 1, 4)):
            assert scratch <= 192, (key, r)
        else:
            assert scratch == 0, (key, r)
    multi = [r for n, r in rep.items() if "rollout_multi_kernel" in n]
    assert multi and all(r["ScratchSize [bytes/lane]"] == 0 for r in multi)
