"""The per-phase profiling build finds every phase mark in the current kernel
source (host only: the instrumented text, no compilation)."""
import os

from paper_2502_11129_amd import phase_profile as P

HDR = os.path.join(os.path.dirname(P.__file__), "csrc", "rollout_kernel.hpp")


def test_every_phase_and_sub_phase_mark_is_found():
    with open(HDR) as f:
        src = f.read()
    s = P.instrument(src)
    assert s.count("s_memtime") == 8 + 7 + 4   # 7 phases + the step's end; 6 tree sub-phases + their end;
    #                                              3 sweep sub-phases + their end
    assert s.count("_ph[") >= 7 and s.count("_sub[") >= 6
    assert "static __device__ unsigned long long g_phase[24][8];" in s
    assert s.count("_pgs[") >= 3
    # the plain source is untouched
    assert "s_memtime" not in src


def test_sweep_part_clocks_close_inside_every_sweep():
    """The Gauss-Seidel parts are clocked in every sweep: the clamp rows'
    clock opens each sweep, so the overflow part's closing clock must sit
    inside the sweep loop's body (after the overflow contacts, before the
    loop's closing brace), not after the loop, where it would charge the
    last sweep's overflow contacts only."""
    with open(HDR) as f:
        src = f.read()
    s = P.instrument(src)
    i_sweep = s.index("for (int sweep = 0; sweep < P.K; ++sweep) {")
    i_close = s.index("_pgs[2] += ")
    i_phase = s.index("_ph[5] += ")          # the Gauss-Seidel phase ends after the loop
    assert i_sweep < i_close < i_phase
    # between the overflow clock and the end of the phase only the loop's
    # closing brace remains
    between = s[s.index("\n", i_close) + 1:s.rindex("\n", 0, i_phase)]
    assert between.strip() == "}"
