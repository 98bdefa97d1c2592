"""The vector-ALU probe that the bench reports beside the published peaks:
a measured FP64 and (unpacked) FP32 fused multiply-add rate, positive and
below the published MI355X vector peaks (FP64 78.6, packed FP32 157.3
TFLOP/s) with 10 % of margin for the clock."""
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")


def test_valu_probe_is_plausible():
    t64 = E.ec_valu_probe(E.EC_FP64)
    t32 = E.ec_valu_probe(E.EC_FP32)
    say(f"case vector-ALU probe: FP64 {t64:.2f} TFLOP/s, FP32 (unpacked) {t32:.2f} TFLOP/s")
    assert 5.0 < t64 < 1.1 * 78.6
    assert 5.0 < t32 < 1.1 * 157.3
    with pytest.raises(E.EcError):
        E.ec_valu_probe(E.EC_BF16X3)
