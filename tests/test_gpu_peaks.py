"""Measured arithmetic peaks (dd_probe_peaks).  The probe is a measurement,
not a result with an exact value, so the test checks what must hold on any
working device: every rate positive and finite, the launch times of the
sizes the probe runs, and the rates below what the unit counts allow at the
clock the runtime reports (a rate above that would mean the compiler folded
the chains away).  Per compute unit and clock, the vector units retire at
most 64 FP32 or 64 FP64 fused multiply-adds (4 SIMDs x 16 lanes; packed
FP32 is disabled in this build) and at most 64 transcendental results."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_probe_rates_are_physical():
    from paper_2001_10986_amd import dd
    pk = dd.probe_peaks()
    cus, mhz = pk["compute_units"], pk["clock_mhz"]
    assert cus > 0 and mhz > 0
    for k in ("fp32_fma_tflops", "fp64_fma_tflops", "exp_f32_per_s", "ms_fp32", "ms_fp64",
              "ms_exp"):
        assert math.isfinite(pk[k]) and pk[k] > 0, (k, pk)
    # upper bounds from the unit counts (10 % slack for the clock the
    # runtime reports against the one the kernels ran at)
    fma_cap = cus * 64 * 2 * mhz * 1e6 / 1e12 * 1.1
    assert pk["fp32_fma_tflops"] <= fma_cap, pk
    assert pk["fp64_fma_tflops"] <= fma_cap, pk
    assert pk["exp_f32_per_s"] <= cus * 64 * mhz * 1e6 * 1.1, pk
    # and a floor far below any working device (one tenth of a percent of
    # the cap), so that a probe that measured nothing fails
    assert pk["fp32_fma_tflops"] >= fma_cap * 1e-3, pk
    assert pk["exp_f32_per_s"] >= cus * 64 * mhz * 1e6 * 1e-3, pk
