"""Device-ceiling probes of the library (FP32 FMA loop, device copy): they run through
the C-ABI and return plausible MI355X figures."""
import pytest

import paper_2204_07137_amd as P

pytestmark = pytest.mark.gpu


def test_probe_ceilings_plausible():
    c = P.probe_ceilings(copy_bytes=256 << 20)
    # non-packed FP32 VALU peak is 78.6 TFLOP/s (256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz)
    assert 10.0 < c["fp32_valu_tflops"] < 90.0, c
    # HBM3E peak 8 TB/s (read + write counted)
    assert 500.0 < c["copy_gbs"] < 10000.0, c
