"""The library's probe kernels (measured denominators for the rooflines)
run and report rates within reach of the chip's published peaks."""
import pytest

from paper_1704_03767_amd import ktau as K

pytestmark = pytest.mark.gpu


def test_probe_kernels_run_and_measure_plausible_peaks():
    # the diagnostics the bench uses for measured denominators
    r = K.probe_peaks(blocks=512, valu_iters=2000, lds_iters=200)
    assert 1e12 < r["valu_lane_ops_per_s"] < 1.5 * 256 * 64 * 2.4e9
    # 128 B per cycle per CU is the older CDNA width; gfx950 reads more
    assert 1e12 < r["lds_bytes_per_s"] < 3.0 * 256 * 128 * 2.4e9
    # each instruction kind of the issue probe: at most one wave instruction
    # per SIMD and cycle (1024 SIMDs; 2.6 GHz leaves room for the clock)
    for name in K.ISSUE_KINDS:
        rate = r["issue_wave_instr_per_s"][name]
        assert 1e10 < rate < 1024 * 2.6e9, (name, rate)
