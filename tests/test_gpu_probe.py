"""Peak probes on the GPU: plausible rates for MI355X (FP32 FMA issue without
packed instructions near 78.6 TFLOP/s, BF16 MFMA below the 2.5 PFLOP/s dense
peak, copy below the 8 TB/s HBM peak) and an exact copy; and the rollout
kernel's sine and cosine against FP64."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_probes_report_plausible_peaks():
    from paper_2502_11129_amd import probe
    fp32 = probe.fp32_fma(blocks=2048, iters=256, reps=2)
    mfma = probe.bf16_mfma(blocks=2048, iters=128, reps=2)
    gbs = probe.copy(nbytes=256 << 20, reps=2)
    print(f"fp32 {fp32:.1f} TFLOP/s, bf16 mfma {mfma:.1f} TFLOP/s, copy {gbs:.0f} GB/s", flush=True)
    sys.stdout.flush()
    assert 5.0 < fp32 < 170.0
    assert 50.0 < mfma < 2700.0
    assert 200.0 < gbs < 9000.0


def test_kernel_sine_cosine_against_fp64():
    """The sine and cosine the rollout kernel uses for joint angles and CPG
    phases, evaluated on the GPU over the angles it sees (|x| <= 10, the
    reduced phases in [0, 2 pi), multiples of pi/4 where the quadrant
    switches, their float neighbours) and up to |x| = 100, against FP64 sin
    and cos of the same float32 inputs: within one float32 ulp at 1
    (1.2e-7) and sin^2 + cos^2 within 3e-7 of 1."""
    import numpy as np
    import torch
    from paper_2502_11129_amd import probe
    x = np.concatenate([np.linspace(-10, 10, 1 << 21), np.linspace(0, 2 * np.pi, 1 << 18),
                        np.arange(-64, 65) * (np.pi / 4), np.linspace(-100, 100, 1 << 18)]).astype(np.float32)
    x = np.concatenate([x, np.nextafter(x, np.float32(np.inf)), np.nextafter(x, np.float32(-np.inf))])
    print(f"[sincos] {x.size} inputs", flush=True)
    sn, cs = probe.sincos(torch.from_numpy(x).cuda())
    sn, cs = sn.cpu().numpy().astype(np.float64), cs.cpu().numpy().astype(np.float64)
    xd = x.astype(np.float64)
    es, ec = np.abs(sn - np.sin(xd)).max(), np.abs(cs - np.cos(xd)).max()
    en = np.abs(sn * sn + cs * cs - 1.0).max()
    print(f"  max abs error sin {es:.3e}, cos {ec:.3e}; |s^2 + c^2 - 1| {en:.3e}", flush=True)
    assert es <= 1.2e-7 and ec <= 1.2e-7
    assert en <= 3e-7
