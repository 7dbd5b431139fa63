"""The microbenchmarks behind the measured ceilings: each returns a rate
between a loose floor and the part's published peak for its unit (MI355X:
256 CUs at 2.4 GHz; FP32 157.3 TFLOP/s with packed FP32, 78.6 without;
FP64 78.6 TFLOP/s; LDS 256 B per clock per CU, 157.3 TB/s)."""
from __future__ import annotations

import pytest

PEAK_FP32 = 157.3e12
PEAK_FP64 = 78.6e12
PEAK_LDS = 256 * 256 * 2.4e9
LANE_CLOCKS = 64 * 256 * 2.4e9  # one result per lane per clock


@pytest.mark.gpu
def test_probes_measure_plausible_ceilings():
    import paper_1907_11678_amd as semb
    f32, ms32 = semb.probe("fma_f32", reps=3)
    f64, _ = semb.probe("fma_f64", reps=3)
    rsq, _ = semb.probe("rsq_f64", reps=3)
    lds, _ = semb.probe("lds_read", reps=3)
    lds2, _ = semb.probe("lds_read2", reps=3)
    print(f"fp32 FMA {f32 / 1e12:.1f} TFLOP/s ({ms32:.2f} ms), fp64 FMA {f64 / 1e12:.1f} TFLOP/s, "
          f"rsq_f64 {rsq / 1e12:.2f} T/s, LDS {lds / 1e12:.1f} TB/s (16-byte reads), "
          f"{lds2 / 1e12:.1f} TB/s (paired 4-byte reads)", flush=True)
    # plain FMAs cannot pass the packed-FP32 peak; a working probe is far above a quarter of it
    assert 0.25 * PEAK_FP32 < f32 < 1.05 * PEAK_FP32
    assert 0.1 * PEAK_FP64 < f64 < 1.05 * PEAK_FP64
    assert 0.01 * LANE_CLOCKS < rsq < 1.05 * LANE_CLOCKS
    assert 0.2 * PEAK_LDS < lds < 1.05 * PEAK_LDS
    assert 0.1 * PEAK_LDS < lds2 < 1.05 * PEAK_LDS
    assert ms32 > 0.5  # long enough to time with events
