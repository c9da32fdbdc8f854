"""CPU/GPU split policy (paper Sec. 6), host only: the allocation rules of the
C ABI on scripted latency curves, against closed forms."""
import numpy as np
import pytest

from paper_2502_11129_amd import sim as S


@pytest.mark.parametrize("n, rg, rc", [(10000, 5000.0, 1000.0), (777, 123.0, 456.0), (32768, 2.0e4, 3.0e3)])
def test_linear_rates_both_rules_give_the_inverse_time_share(n, rg, rc):
    # GPU time m / rg through the origin, host time h / rc: balance at h = n rc / (rg + rc)
    pts = np.array([n // 16, n // 4, n], np.int32)
    r = S.split_allocation(n, pts, pts / rg, 1.0 / rc)
    h_exact = n * rc / (rg + rc)
    assert abs(r["n_host_paper"] - h_exact) <= 0.5 + 1e-9
    assert abs(r["n_host_makespan"] - h_exact) <= 1.0
    # both makespans equal the balanced time up to one variant's worth
    t_bal = (n - h_exact) / rg
    assert abs(r["makespan_opt_s"] - t_bal) <= 1.0 / min(rg, rc)
    assert r["makespan_opt_s"] <= r["makespan_paper_s"] + 1e-12


def test_flat_then_linear_curve_closed_form():
    # GPU: 1 s flat up to 1000 variants, then 1 ms per variant; host 10 ms per variant; n = 5000.
    # Balance of (5000 - h) / 1000 = h / 100 at h = 454.5: h = 454 gives max(4.546, 4.54) = 4.546.
    r = S.split_allocation(5000, [1000, 5000], [1.0, 5.0], 0.01)
    assert r["n_host_makespan"] == 454
    assert abs(r["makespan_opt_s"] - 4.546) < 1e-12
    assert r["n_host_paper"] == 455           # round(5000 * 5 / 55)


def test_flat_region_makes_the_rules_differ():
    # GPU saturates only above 4000 variants: every host share in [1000, 1500]
    # gives the 3 s floor; the makespan rule takes the smallest such share.
    r = S.split_allocation(5000, [4000, 5000], [3.0, 3.5], 0.002)
    assert r["n_host_makespan"] == 1000 and r["makespan_opt_s"] == 3.0
    assert r["n_host_paper"] == round(5000 * 3.5 / 13.5)
    assert r["makespan_paper_s"] == 3.0


def test_host_share_zero_when_the_host_is_slow_and_all_when_the_gpu_is_slow():
    r = S.split_allocation(1000, [1000], [0.1], 10.0)
    assert r["n_host_makespan"] == 0 and r["n_host_paper"] == 0
    r = S.split_allocation(1000, [1000], [1e6], 1e-9)
    assert r["n_host_makespan"] == 1000 and r["n_host_paper"] == 1000


def test_makespan_rule_is_optimal_on_a_scripted_curve():
    """Brute force over every host share with an independent evaluation of a
    scripted concave-then-linear curve (sampled exactly at its knots)."""
    n = 3000
    knots = np.array([100, 500, 1000, 2000, 3000], np.int32)
    times = np.array([0.40, 0.45, 0.55, 0.95, 1.45])
    host = 1.3e-3
    r = S.split_allocation(n, knots, times, host)

    def t_gpu(m):
        if m == 0:
            return 0.0
        return float(np.interp(m, knots, times)) if m <= knots[-1] else None

    best = min(max(t_gpu(n - h), h * host) for h in range(n + 1))
    assert abs(r["makespan_opt_s"] - best) < 1e-12
    h = r["n_host_makespan"]
    assert abs(max(t_gpu(n - h), h * host) - best) < 1e-12


@pytest.mark.parametrize("args", [
    (100, [], [], 1.0),
    (100, [50, 40], [1.0, 2.0], 1.0),
    (100, [50], [1.0], 0.0),
    (100, [0], [1.0], 1.0),
    (-1, [50], [1.0], 1.0),
])
def test_invalid_inputs(args):
    with pytest.raises(S.SimError) as e:
        S.split_allocation(*args)
    assert e.value.code == S.SIM_E_INVALID and len(str(e.value)) > 10
