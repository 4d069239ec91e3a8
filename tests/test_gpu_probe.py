"""Device throughput probes (measurement support, not part of the method):
each returns a rate within what an MI355X can physically reach."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_rates_are_plausible():
    from paper_1409_8186_amd import probe
    fma = probe("fp64_fma")
    mfma = probe("fp64_mfma")
    copy = probe("copy", 256 << 20)
    print(f"fp64 fma {fma:.1f} TFLOP/s, fp64 mfma {mfma:.1f} TFLOP/s, copy {copy:.0f} GB/s")
    # published dense peaks: 78.6 TFLOP/s for both; HBM 8 TB/s
    assert 5.0 < fma < 90.0
    assert 5.0 < mfma < 90.0
    assert 200.0 < copy < 9000.0
