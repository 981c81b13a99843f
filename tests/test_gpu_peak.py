"""The peak probes of fpm_peak.h run on the MI355X and land near the
published figures the roofline is priced against (3.93e13 int-VALU lane-ops/s
for the vector filter's instruction mix, 5.0e15 dense int8 matrix ops/s);
the bounds are loose (clock and power states vary), the numbers themselves
are reported by the benchmark."""
import pytest

pytestmark = pytest.mark.gpu


def test_peaks_are_measured(gpu):
    from paper_1711_08475_amd import fpm

    print("[case] peak probes", flush=True)
    p = fpm.fpm_measure_peaks()
    print(p, flush=True)
    assert p["compute_units"] > 0
    assert p["valu_ms"] > 0 and p["matrix_ms"] > 0
    assert p["valu_ops"] == p["compute_units"] * 8 * 256 * 8192 * 96
    assert p["matrix_ops"] == p["compute_units"] * 8 * 4 * 2 * 16384 * 65536
    assert 0.4 * 3.93e13 < p["int_valu_ops_per_s"] < 1.3 * 3.93e13
    assert 0.2 * 5.0e15 < p["int8_matrix_ops_per_s"] < 1.3 * 5.0e15
