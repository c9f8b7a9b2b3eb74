"""Measured peaks (diagnostic entry points used beside the published peaks in the roofline
figures): the FP32 FMA loop and the device copy return rates in a physically possible range."""
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def test_peak_fp32_and_copy_rates():
    import paper_1212_1095_amd as vor
    say("peaks: FMA loop, 256 MiB copy")
    fma = vor.vor_peak_fp32(0)
    # non-packed FP32 FMA: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x clock (at most 2.4 GHz)
    assert 5.0 < fma < 1.05 * 78.7
    copy = vor.vor_peak_copy(256 << 20, 0)
    assert 100.0 < copy < 1.05 * 8000.0 * 1.5   # read plus written; L2/MALL may add a little


def test_peak_copy_rejects_tiny_size():
    import paper_1212_1095_amd as vor
    with pytest.raises(vor.VorError) as e:
        vor.vor_peak_copy(8, 0)
    assert e.value.status == vor.VOR_E_INVAL
