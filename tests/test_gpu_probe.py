"""Peak probes on the GPU: plausible rates for MI355X (FP32 FMA issue without
packed instructions near 78.6 TFLOP/s, BF16 MFMA below the 2.5 PFLOP/s dense
peak, copy below the 8 TB/s HBM peak) and an exact copy."""
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
